"""GPU parity of long systems (tri n > 2048, penta n > 1024): the three-launch
path (reduce, scan, solve; the solution array as scratch) against the FP64
oracle through the C ABI -- solves and adjoint solves, tri and penta,
periodic or not, full and ragged last chunks, every chunk size, small and
large batches, strided arrays; and the long Cahn-Hilliard step against the
oracle's step."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2107_05395_amd import BandBatchError, Factor, inputs
from tests.gpu_util import dev, fp64_tol, host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    from paper_2107_05395_amd import solver  # noqa: F401
    oracle.build()


def _make(kind, n, seed, cyclic):
    if kind == "tri":
        bands = inputs.random_dominant_tri(n, seed)
        return Factor.tri(*bands, cyclic=cyclic), bands
    bands = inputs.random_dominant_penta(n, seed)
    return Factor.penta(*bands, cyclic=cyclic), bands


def _oracle(kind, bands, rhs, cyclic, adjoint):
    if kind == "tri":
        fn = oracle.tri_adjoint if adjoint else oracle.tri_solve
    else:
        fn = oracle.penta_adjoint if adjoint else oracle.penta_solve
    return fn(*bands, rhs, cyclic=cyclic)


CASES = [("tri", 2049, 70), ("tri", 4096, 64), ("tri", 8192, 1), ("tri", 5000, 200),
         ("tri", 16384, 3), ("penta", 1025, 65), ("penta", 4096, 33), ("penta", 8192, 64),
         ("penta", 3001, 129), ("penta", 16384, 2)]


@pytest.mark.parametrize("kind,n,m", CASES)
@pytest.mark.parametrize("cyclic", [False, True])
@pytest.mark.parametrize("adjoint", [False, True])
def test_long_solves_match_oracle(kind, n, m, cyclic, adjoint):
    say("long", kind, n, m, "cyclic" if cyclic else "", "adjoint" if adjoint else "")
    f, bands = _make(kind, n, seed=n + m + cyclic, cyclic=cyclic)
    assert f.plan(m)["scalar"]
    rhs = inputs.uniform_batch(n, m, seed=3 * n + m)
    out = f.adjoint(dev(rhs)) if adjoint else f.solve(dev(rhs))
    err = rel_err(host(out), _oracle(kind, bands, rhs, cyclic, adjoint))
    say("  rel err", err)
    assert err < 1e-12


@pytest.mark.parametrize("chunk", ["16", "32", "64"])
@pytest.mark.parametrize("kind,n", [("tri", 4097), ("penta", 2050), ("penta", 2048)])
def test_long_chunk_sizes(chunk, kind, n, tuning):
    tuning.set("max_chunk", chunk)
    for cyclic in (False, True):
        f, bands = _make(kind, n, seed=n + int(chunk), cyclic=cyclic)
        assert f.plan(100)["chunk"] == int(chunk)
        rhs = inputs.uniform_batch(n, 100, seed=n)
        err = rel_err(host(f.solve(dev(rhs))), _oracle(kind, bands, rhs, cyclic, False))
        say("long chunk", chunk, kind, n, cyclic, err)
        assert err < 1e-12


@pytest.mark.parametrize("kind,n,m", [("tri", 2049, 1), ("tri", 8192, 65), ("tri", 5000, 300),
                                      ("penta", 1025, 1), ("penta", 4096, 64), ("penta", 3001, 129)])
@pytest.mark.parametrize("cyclic", [False, True])
@pytest.mark.parametrize("adjoint", [False, True])
def test_long_scan_variants_match(kind, n, m, cyclic, adjoint, tuning):
    """The two scans of a long solve -- one lane per system stepping through
    its chunks, and one wave per system scanning 64 chunks' affine maps at a
    time -- each against the oracle, and against each other (they differ
    only in how the chunk-boundary recurrences are rounded)."""
    say("long scans", kind, n, m, cyclic, adjoint)
    f, bands = _make(kind, n, seed=2 * n + m, cyclic=cyclic)
    rhs = dev(inputs.uniform_batch(n, m, seed=5 * n + m))
    ref = _oracle(kind, bands, host(rhs), cyclic, adjoint)
    outs = []
    for spread in (0, 1):
        tuning.set("long_spread", spread)
        outs.append(host(f.adjoint(rhs) if adjoint else f.solve(rhs)))
        err = rel_err(outs[-1], ref)
        say("  spread", spread, err)
        assert err < 1e-12
    assert rel_err(outs[0], outs[1]) < 1e-13


def test_long_large_batch_sampled():
    """A batch of 2^16 + 5 systems (1 GiB per array at n = 2048 penta): the
    large-batch chunk size, every 64-system group and the batch tail, checked
    on sampled systems."""
    n, m = 2048, (1 << 16) + 5
    f, bands = _make("penta", n, seed=5, cyclic=True)
    assert f.plan(m)["chunk"] == 64
    rhs = inputs.uniform_batch(n, m, seed=6)
    out = f.solve(dev(rhs))
    cols = np.unique(np.r_[np.linspace(0, m - 1, 400).astype(np.int64), m - 1, m - 2, 64, 63])
    err = rel_err(host(out[:, cols]), _oracle("penta", bands, rhs[:, cols], True, False))
    say("long large batch", err)
    assert err < 1e-12


def test_long_strided_and_untouched_columns():
    """ld > m: a column slice of a wider array; the columns past m of both
    the input and the output (which serves as scratch) are left alone."""
    n, m, extra = 3000, 150, 21
    f, bands = _make("tri", n, seed=9, cyclic=True)
    rhs = inputs.uniform_batch(n, m, seed=10)
    wide_in = torch.full((n, m + extra), 7.0, dtype=torch.float64, device="cuda")
    wide_out = torch.full((n, m + extra), 9.0, dtype=torch.float64, device="cuda")
    wide_in[:, :m] = dev(rhs)
    f.solve(wide_in[:, :m], out=wide_out[:, :m])
    assert rel_err(host(wide_out[:, :m]), _oracle("tri", bands, rhs, True, False)) < 1e-12
    assert torch.all(wide_out[:, m:] == 9.0) and torch.all(wide_in[:, m:] == 7.0)
    assert np.array_equal(host(wide_in[:, :m]), rhs)


@pytest.mark.parametrize("kind,n,m,cyclic", [("tri", 4096, 70, False), ("tri", 8192, 5000, True),
                                             ("penta", 2048, 65, True), ("penta", 8192, 9000, False)])
def test_long_f32_rhs_f64(kind, n, m, cyclic):
    """FP32 right-hand-side data on long systems, solved in FP64: against the
    oracle on the promoted values at 1e-12, and bitwise the FP64 solve of
    the promoted array (same three launches and arithmetic); adjoint too."""
    say("long f32rhs_f64", kind, n, m, cyclic)
    f, bands = _make(kind, n, seed=n + 7, cyclic=cyclic)
    r32 = inputs.uniform_batch(n, m, seed=5 * n + m).astype(np.float32)
    t = dev(r32, torch.float32)
    x = f.solve(t, precision="f32rhs_f64")
    assert rel_err(host(x), _oracle(kind, bands, r32.astype(np.float64), cyclic, False)) < 1e-12
    assert torch.equal(x, f.solve(t.double()))
    assert torch.equal(f.adjoint(t, precision="f32rhs_f64"), f.adjoint(t.double()))


def test_long_rejects_in_place_and_other_precisions():
    n = 4096
    f, _ = _make("tri", n, seed=1, cyclic=False)
    t = dev(inputs.uniform_batch(n, 10, seed=2))
    with pytest.raises(BandBatchError):
        f.solve(t, out=t)
    with pytest.raises(BandBatchError):
        f.solve(t, precision="f32r")


@pytest.mark.parametrize("n,m", [(2048, 100), (4096, 70), (8192, 3), (3000, 64), (2048, 8195)])
def test_long_cahn_hilliard_steps_match_oracle(n, m):
    """The Section 5.1 step of long periodic systems (right-hand side formed
    inside the launches from the state and its neighbour rows), two steps
    ping-ponged, against the oracle's steps; dt = 0.1 dx, L = 2 pi."""
    L, gamma = 2 * math.pi, 0.01
    dx = L / n
    dt = 0.1 * dx
    f = Factor.cahn_hilliard(n, L, gamma, dt)
    sigma, alpha = oracle.ch_coefficients(gamma, dx, dt)
    c0 = 0.3 + inputs.uniform_batch(n, m, seed=n + m, lo=-0.1, hi=0.1)
    a, b = dev(c0), torch.empty(n, m, dtype=torch.float64, device="cuda")
    f.ch_step(a, f.alpha, out=b)
    f.ch_step(b, f.alpha, out=a)
    ref = oracle.ch_step(c0, sigma, alpha, steps=2)
    err = rel_err(host(a), ref)
    tol = fp64_tol(1.0 + 16.0 * sigma, 2)
    say("long CH", n, m, err, "tol", tol)
    assert err < tol


@pytest.mark.parametrize("n,m", [(2048, 100), (3001, 70), (4096, 64), (8192, 5)])
def test_long_forced_steps_match_oracle(n, m):
    """The forced travelling-wave step of long periodic systems (WENO
    advection and forcing formed inside the launches from the state and three
    halo rows on each side), per-run v of both signs and zero, f0 and k
    varying, two steps ping-ponged, against the oracle's steps; dt = 0.1 dx."""
    L, gamma = 2 * math.pi, 0.01
    dx = L / n
    dt = 0.1 * dx
    g = inputs.rng(n + m)
    v = g.uniform(-1, 1, m)
    v[::5] = 0.0
    f0 = g.uniform(0, 2, m)
    k = g.integers(1, 4, m).astype(np.float64) * (2 * math.pi / L)
    c0 = g.uniform(0, 1.5, m) + inputs.uniform_batch(n, m, seed=n + 2 * m, lo=-0.1, hi=0.1)
    f = Factor.cahn_hilliard(n, L, gamma, dt)
    assert f.long
    a, b = dev(c0), torch.empty(n, m, dtype=torch.float64, device="cuda")
    pv, pf, pk = dev(v), dev(f0), dev(k)
    f.ch_forced_step(a, dt, dx, pv, pf, pk, out=b)
    f.ch_forced_step(b, dt, dx, pv, pf, pk, out=a)
    sigma, alpha = oracle.ch_coefficients(gamma, dx, dt)
    beta, amp, kdx = oracle.ch_forced_parameters(dt, dx, v, f0, k)
    ref = oracle.ch_forced_step(c0, sigma, alpha, beta, amp, kdx, steps=2)
    err = rel_err(host(a), ref)
    tol = fp64_tol(1.0 + 16.0 * sigma, 2)
    say("long forced CH", n, m, err, "tol", tol)
    assert err < tol


def test_long_forced_run_alternates_buffers():
    """Factor.ch_forced_run on a long system: several one-step calls, the
    input left unchanged, the result equal to the same calls made by hand."""
    n, m = 2050, 40
    L = 2 * math.pi
    dx = L / n
    dt = 0.1 * dx
    f = Factor.cahn_hilliard(n, L, 0.01, dt)
    c0 = dev(0.5 + inputs.uniform_batch(n, m, seed=4, lo=-0.1, hi=0.1))
    keep = c0.clone()
    pv = torch.full((m,), 0.5, dtype=torch.float64, device="cuda")
    pf = torch.full((m,), 1.0, dtype=torch.float64, device="cuda")
    pk = torch.full((m,), 1.0, dtype=torch.float64, device="cuda")
    out = f.ch_forced_run(c0, dt, dx, pv, pf, pk, steps=3)
    x = c0
    for _ in range(3):
        x = f.ch_forced_step(x, dt, dx, pv, pf, pk, out=torch.empty_like(x))
    assert torch.equal(out, x) and torch.equal(c0, keep)


@pytest.mark.parametrize("kind,n,m", [("tri", 2049, 70), ("tri", 5000, 3), ("penta", 1025, 65),
                                      ("penta", 3001, 129), ("penta", 8192, 1),
                                      ("tri", 2100, 8193)])
@pytest.mark.parametrize("cyclic", [False, True])
def test_long_cn_steps_match_oracle(kind, n, m, cyclic):
    """Crank-Nicolson steps A c' = B c of long systems (the stencil formed
    inside the launches from the state and K halo rows on each side, wrapped
    or zero): one step per call and a 3-step trajectory against the oracle's
    steps; a random non-symmetric stencil on row-dependent bands."""
    say("long CN", kind, n, m, cyclic)
    f, bands = _make(kind, n, seed=3 * n + m, cyclic=cyclic)
    g = inputs.rng(n + m)
    w = list(g.uniform(-1, 1, 3 if kind == "tri" else 5))
    c0 = inputs.uniform_batch(n, m, seed=n + 7 * m)
    one = f.cn_step(dev(c0), w, steps=1)
    ref1 = oracle.cn_step(bands, w, c0, steps=1, cyclic=cyclic)
    assert rel_err(host(one), ref1) < 1e-12
    traj = f.cn_trajectory(dev(c0), w, 3)
    assert torch.equal(traj[0], one)
    ref = c0
    for s in range(3):
        ref = oracle.cn_step(bands, w, ref, steps=1, cyclic=cyclic)
        assert rel_err(host(traj[s]), ref) < 1e-12, s


@pytest.mark.parametrize("kind,cyclic", [("tri", False), ("penta", True)])
def test_long_adjoint_trajectory(kind, cyclic):
    """bb_adjoint_trajectory on long systems: repeated transposed solves with
    the factor's own factorisation, against the oracle's."""
    n, m = (4097, 40) if kind == "tri" else (2000, 40)
    f, bands = _make(kind, n, seed=n, cyclic=cyclic)
    gh = inputs.uniform_batch(n, m, seed=2 * n)
    traj = f.adjoint_trajectory(dev(gh), 4)
    lam = gh
    for s in range(4):
        lam = _oracle(kind, bands, lam, cyclic, True)
        assert rel_err(host(traj[s]), lam) < 1e-12, s


def test_long_rollout_gradients_match_oracle():
    """The checkpointed rollout and its gradients on a long system
    (n = 3000 > 2048): forward steps, recomputation and adjoint trajectories
    all through the long-system launches; against the oracle's recursion."""
    from paper_2107_05395_amd import banded_rollout, mse_loss
    n, m, steps, r = 3000, 50, 7, 0.5
    g = inputs.rng(11)
    D = g.uniform(0.5, 1.5, n)
    u0 = inputs.uniform_batch(n, m, seed=12)
    target = inputs.uniform_batch(n, m, seed=13)
    Dt = torch.tensor(D, dtype=torch.float64, requires_grad=True)
    u0t = dev(u0).requires_grad_(True)
    uT = banded_rollout(u0t, (-r * Dt, 1 + 2 * r * Dt, -r * Dt), steps=steps, checkpoint_every=3)
    loss = mse_loss(uT, dev(target))
    loss.backward()
    ref_loss, ref_dD, ref_du0 = oracle.diffusion_loss_and_grads(D, r, u0, target, steps)
    assert abs(loss.item() - ref_loss) <= 1e-12 * abs(ref_loss)
    assert rel_err(host(u0t.grad), ref_du0) < 1e-12
    assert np.max(np.abs(Dt.grad.numpy() - ref_dD)) <= 1e-12 * np.max(np.abs(ref_dD))
