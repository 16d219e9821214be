"""GPU parity of the fused forced Cahn-Hilliard steps in the frame of the
travelling wave (per-run advection speed and forcing, HJ-WENO5 advection)
against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2107_05395_amd import inputs
from tests.gpu_util import dev, fp64_tol, host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    from paper_2107_05395_amd import solver  # noqa: F401
    oracle.build()


def _setup(n, m, seed, L=2 * math.pi):
    """Flow-pattern style batch: dt = 0.1 dx, gamma = 0.01; per run a speed
    v in [-1, 1] (some exactly 0), amplitude f0 in [0, 2], wavenumber k in
    {1, 2, 3}, mean concentration in [0, 1.5] plus U[-0.1, 0.1).  The GPU side
    gets the physical parameters and the product's factor; the oracle side
    maps them with its own coefficients."""
    from paper_2107_05395_amd import Factor
    dx = L / n
    dt = 0.1 * dx
    g = inputs.rng(seed)
    v = g.uniform(-1, 1, m)
    v[::7] = 0.0
    f0 = g.uniform(0, 2, m)
    k = g.integers(1, 4, m).astype(np.float64) * (2 * math.pi / L)
    mean = g.uniform(0, 1.5, m)
    c0 = mean + inputs.uniform_batch(n, m, seed=seed + 1, lo=-0.1, hi=0.1)
    f = Factor.cahn_hilliard(n, L, 0.01, dt)
    sigma, alpha = oracle.ch_coefficients(0.01, dx, dt)
    beta, amp, kdx = oracle.ch_forced_parameters(dt, dx, v, f0, k)
    gpu = dict(dt=dt, dx=dx, v=dev(v), f0=dev(f0), k=dev(k))
    ref = dict(sigma=sigma, alpha=alpha, beta=beta, amp=amp, kdx=kdx)
    return f, c0, gpu, ref


def _oracle_steps(c0, ref, steps, cols=None):
    sel = slice(None) if cols is None else cols
    return oracle.ch_forced_step(c0[:, sel], ref["sigma"], ref["alpha"], ref["beta"][sel],
                                 ref["amp"][sel], ref["kdx"][sel], steps=steps)


def _gpu_steps(f, c, gpu, steps, out=None):
    return f.ch_forced_step(c, gpu["dt"], gpu["dx"], gpu["v"], gpu["f0"], gpu["k"], steps=steps,
                            out=out)


@pytest.mark.parametrize("n,m", [(256, 300), (512, 300), (64, 300), (1024, 300), (300, 200),
                                 (1000, 100), (7, 50), (5, 40), (256, (1 << 16) + 3),
                                 (64, 70000)])
def test_forced_steps_match_oracle(n, m):
    """One step at every size (the Cahn-Hilliard matrix of dt = 0.1 dx has
    kappa = 1 + 16 sigma: 1.1e3 at n = 256, 8.7e3 at 512, 6.9e4 at 1024, which
    sets the FP64 tolerance above 1e-12 from n = 512 on), then five steps."""
    say("forced", n, m)
    f, c0, gpu, ref = _setup(n, m, seed=n + m)
    kappa = 1.0 + 16.0 * ref["sigma"]
    cols = np.unique(np.r_[np.linspace(0, m - 1, 300).astype(np.int64), m - 1])
    for steps in (1, 5):
        want = _oracle_steps(c0, ref, steps, cols)
        out = host(_gpu_steps(f, dev(c0), gpu, steps))
        err = rel_err(out[:, cols], want)
        say("  steps", steps, "rel err", err, "tol", fp64_tol(kappa, steps))
        assert err < fp64_tol(kappa, steps)


@pytest.mark.parametrize("n", [64, 256, 512, 1024])
def test_forced_kernel_variants_agree_bitwise(n, tuning):
    """Scalar coefficients with one chunk per wave, the LDS split group and
    the LDS one-wave group do the same arithmetic (64-row chunks forced)."""
    tuning.set("max_chunk", "64")
    m = 3000
    f, c0, gpu, ref = _setup(n, m, seed=7 * n)
    t = dev(c0)
    a = host(_gpu_steps(f, t, gpu, 4))
    tuning.set("ch_uniform", "0")
    assert np.array_equal(a, host(_gpu_steps(f, t, gpu, 4)))
    tuning.set("waves_per_system", "1")
    assert np.array_equal(a, host(_gpu_steps(f, t, gpu, 4)))


@pytest.mark.parametrize("chunk", ["4", "8", "16", "32"])
def test_forced_chunk_sizes_match_oracle(chunk, tuning):
    tuning.set("max_chunk", chunk)
    for n in (256, 250):
        f, c0, gpu, ref = _setup(n, 130, seed=11 + n)
        want = _oracle_steps(c0, ref, 3)
        out = host(_gpu_steps(f, dev(c0), gpu, 3))
        assert rel_err(out, want) < 1e-12, (n, chunk)


def test_forced_without_forcing_matches_plain_steps_and_in_place():
    n, m = 256, 500
    f, c0, gpu, ref = _setup(n, m, seed=3)
    z = torch.zeros(m, dtype=torch.float64, device="cuda")
    t = dev(c0)
    a = host(f.ch_forced_step(t, gpu["dt"], gpu["dx"], z, z, gpu["k"], steps=6))
    b = host(f.ch_step(t, f.alpha, steps=6))
    assert rel_err(a, b) < 1e-13
    _gpu_steps(f, t, gpu, 6, out=t)
    assert rel_err(host(t), _oracle_steps(c0, ref, 6)) < 1e-12


def test_forced_rejects_bad_parameters():
    f, c0, gpu, ref = _setup(64, 10, seed=4)
    with pytest.raises(ValueError):
        f.ch_forced_step(dev(c0), gpu["dt"], gpu["dx"], gpu["v"][:5], gpu["f0"], gpu["k"])
    from paper_2107_05395_amd import BandBatchError
    with pytest.raises(BandBatchError):
        f.ch_forced_step(dev(c0), -1.0, gpu["dx"], gpu["v"], gpu["f0"], gpu["k"])


def test_steppers_on_strided_batches():
    """ld > m (a column slice of a wider array) for the Crank-Nicolson, the
    Cahn-Hilliard-with-statistic and the forced steps: the same results as
    on contiguous arrays, and the columns past m untouched."""
    n, m, extra = 256, 700, 37
    f, c0, gpu, ref = _setup(n, m, seed=21)
    wide = torch.zeros(n, m + extra, dtype=torch.float64, device="cuda")
    wide[:, :m] = dev(c0)
    wide[:, m:] = 7.0
    out_wide = torch.full_like(wide, 9.0)
    view, oview = wide[:, :m], out_wide[:, :m]
    got = _gpu_steps(f, view, gpu, 4, out=oview)
    want = _gpu_steps(f, dev(c0), gpu, 4)
    assert np.array_equal(host(got), host(want))
    assert torch.all(out_wide[:, m:] == 9.0) and torch.all(wide[:, m:] == 7.0)
    out_wide.fill_(9.0)
    _, lb = f.ch_step_stats(view, f.alpha, steps=4, every=2, out=oview)
    _, lb_ref = f.ch_step_stats(dev(c0), f.alpha, steps=4, every=2)
    assert np.array_equal(host(lb), host(lb_ref)) and torch.all(out_wide[:, m:] == 9.0)
    from paper_2107_05395_amd import Factor
    bands, w = inputs.cn_hyperdiffusion_problem(n, 0.5)
    g = Factor.penta(*bands, cyclic=True)
    out_wide.fill_(9.0)
    got = g.cn_step(view, w, steps=3, out=oview)
    assert np.array_equal(host(got), host(g.cn_step(dev(c0), w, steps=3)))
    assert torch.all(out_wide[:, m:] == 9.0)
