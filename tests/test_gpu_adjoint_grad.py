"""GPU parity of the fused backward of a rollout (bb_adjoint_band_grad): the
adjoints and band gradients over a stretch of implicit steps against the
FP64 oracle's transposed solves and batch reductions, on every geometry of
the fused kernel (coefficients through the scalar cache or staged in LDS;
16, 32 or 64 systems per group; 32- and 64-row chunks; a ragged last group)
and on the step-by-step path (short chunks, long systems)."""
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


def _factor(kind, cyclic, n):
    from paper_2107_05395_amd import Factor
    bands = (inputs.random_dominant_tri(n, seed=n + 1) if kind == "tri"
             else inputs.random_dominant_penta(n, seed=n + 1))
    f = Factor.tri(*bands, cyclic=cyclic) if kind == "tri" else Factor.penta(*bands, cyclic=cyclic)
    return f, bands


def _oracle_backward(kind, cyclic, bands, g, us, grad0):
    """d_{t-1} = A^{-T} d_t from d_T = g, grad += -sum_t d_{t-1} u_t^T (band
    form), and the scale max|d| max|u| m summed over the steps."""
    adj = oracle.tri_adjoint if kind == "tri" else oracle.penta_adjoint
    nb = 3 if kind == "tri" else 5
    d, ref, scale = g, grad0.copy(), 0.0
    for t in range(len(us), 0, -1):
        d = adj(*bands, d, cyclic=cyclic)
        ref += oracle.band_grad(d, us[t - 1], nb, cyclic=cyclic)
        scale += np.max(np.abs(d)) * np.max(np.abs(us[t - 1])) * g.shape[1]
    return d, ref, scale


# kind, cyclic, n, m, steps, tuning, fused: the geometry each case reaches
CASES = [
    ("tri", False, 1024, 20000, 3, {}, True),        # LDS table, 64-row chunks, 32 systems, 8 waves
    ("tri", True, 1024, 20000, 2, {}, True),
    ("penta", False, 1024, 20000, 2, {}, True),
    ("penta", True, 1024, 20000, 3, {}, True),
    ("tri", False, 2048, 4000, 2, {}, True),         # 64-row chunks, 16 systems per group
    ("tri", True, 2048, 2500, 2, {}, True),          # the largest LDS area (158 KB)
    ("tri", False, 1024, 3000, 3, {}, True),         # 32-row chunks, 16 systems
    ("tri", True, 512, 5000, 4, {}, True),           # 32-row chunks, 32 systems
    ("tri", False, 256, 8192, 3, {}, True),          # scalar coefficients, 32-row chunks
    ("tri", False, 64, 70000, 2, {}, True),          # scalar, two chunks per system
    ("penta", False, 512, 20000, 2, {}, True),       # scalar, 64-row chunks
    ("penta", True, 256, 5000, 3, {}, True),         # scalar, 32-row chunks
    ("penta", False, 128, 20000, 2, {}, True),
    ("tri", True, 64, 140000, 2, {}, True),          # one chunk per system, one wave per group
    ("penta", False, 64, 140000, 2, {}, True),
    ("tri", False, 32, 140000, 3, {}, True),         # one 32-row chunk per system
    ("tri", False, 256, 8192, 2, {"ch_uniform": 0}, True),     # LDS table, 4-wave groups
    ("penta", True, 512, 20000, 2, {"ch_uniform": 0}, True),   # LDS table, 4-wave groups
    ("tri", False, 256, 8192, 3, {"ch_uniform": 0, "waves_per_system": 1}, False),
    ("penta", True, 1024, 2000, 2, {}, False),       # 32-row chunks, 16 systems: step by step
    ("tri", False, 64, 33, 3, {}, False),            # small batch, short chunks
    ("penta", True, 7, 33, 2, {}, False),
    ("tri", True, 4096, 300, 3, {}, False),          # long systems
    ("penta", False, 2048, 200, 2, {}, False),
]


@pytest.mark.parametrize("kind,cyclic,n,m,steps,tune,fused", CASES)
def test_adjoint_band_grad_matches_oracle(kind, cyclic, n, m, steps, tune, fused, tuning):
    say("adjoint + band grad", kind, cyclic, n, m, steps, tune)
    for name, value in tune.items():
        tuning.set(name, value)
    f, bands = _factor(kind, cyclic, n)
    assert f.adjoint_band_grad_fused(m) == fused
    g = inputs.uniform_batch(n, m, seed=3 * n + m)
    # the kernel pairs the adjoints with whatever states it is given: random
    # ones check the pairing and the reduction independently of a forward run
    us = [inputs.uniform_batch(n, m, seed=1000 + 7 * t + n) for t in range(steps)]
    grad0 = inputs.uniform_batch(f.nbands, n, seed=5)
    traj = torch.stack([dev(u) for u in us])
    lam, grad = f.adjoint_band_grad(dev(g), traj, dev(grad0))
    d0, ref, scale = _oracle_backward(kind, cyclic, bands, g, us, grad0)
    assert rel_err(host(lam), d0) < 1e-12
    assert np.max(np.abs(host(grad) - ref)) < 1e-13 * scale
    # the adjoints are the adjoint trajectory's, bitwise
    assert torch.equal(lam, f.adjoint_trajectory(dev(g), steps)[-1])
    # the band gradients repeat bitwise (fixed summation order)
    lam2, grad2 = f.adjoint_band_grad(dev(g), traj, dev(grad0))
    assert torch.equal(grad2, grad) and torch.equal(lam2, lam)


@pytest.mark.parametrize("kind,cyclic,n,m", [("tri", True, 1024, 20000), ("penta", False, 256, 5000)])
def test_adjoint_band_grad_paths_agree(kind, cyclic, n, m, tuning):
    """The fused kernel and the step-by-step path (forced by tuning) give the
    same adjoints and band gradients to rounding, and the step-by-step path
    equals bb_adjoint_trajectory followed by bb_band_grad per step bitwise."""
    say("adjoint + band grad paths", kind, cyclic, n, m)
    f, _ = _factor(kind, cyclic, n)
    steps = 3
    g = dev(inputs.uniform_batch(n, m, seed=11))
    traj = torch.stack([dev(inputs.uniform_batch(n, m, seed=20 + t)) for t in range(steps)])
    assert f.adjoint_band_grad_fused(m)
    lam_f, grad_f = f.adjoint_band_grad(g, traj)
    tuning.set("ch_uniform", 0)
    tuning.set("waves_per_system", 1)
    assert not f.adjoint_band_grad_fused(m)
    lam_s, grad_s = f.adjoint_band_grad(g, traj)
    lams = f.adjoint_trajectory(g, steps)
    sep = torch.zeros_like(grad_s)
    for j in range(steps):
        f.band_grad(lams[j], traj[steps - 1 - j], sep)
    assert torch.equal(lam_s, lams[-1]) and torch.equal(grad_s, sep)
    assert rel_err(host(lam_f), host(lam_s)) < 1e-13
    scale = float(torch.max(torch.abs(lams)) * torch.max(torch.abs(traj))) * m * steps
    assert float(torch.max(torch.abs(grad_f - grad_s))) < 1e-13 * scale


def test_adjoint_band_grad_in_place_and_odd_steps(tuning):
    """lam may be g; an odd number of steps on the step-by-step path ends in
    the workspace and is copied out."""
    from paper_2107_05395_amd import _lib
    from paper_2107_05395_amd.solver import check
    import ctypes
    say("adjoint + band grad in place")
    for tune in ({}, {"ch_uniform": 0, "waves_per_system": 1}):
        for name, value in tune.items():
            tuning.set(name, value)
        f, _ = _factor("tri", False, 256)
        n, m, steps = 256, 8192, 3
        gh = inputs.uniform_batch(n, m, seed=31)
        traj = torch.stack([dev(inputs.uniform_batch(n, m, seed=40 + t)) for t in range(steps)])
        want_lam, want_grad = f.adjoint_band_grad(dev(gh), traj)
        buf = dev(gh)
        grad = torch.zeros_like(want_grad)
        nbytes = _lib.lib().bb_adjoint_band_grad_workspace_bytes(f._handle, m, m)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=buf.device)
        torch.cuda.synchronize()
        check(_lib.lib().bb_adjoint_band_grad(f._handle, ctypes.c_void_p(buf.data_ptr()),
                                              ctypes.c_void_p(traj.data_ptr()),
                                              ctypes.c_void_p(buf.data_ptr()), m, m, steps,
                                              ctypes.c_void_p(grad.data_ptr()),
                                              ctypes.c_void_p(ws.data_ptr()), nbytes, None))
        torch.cuda.synchronize()
        assert torch.equal(buf, want_lam) and torch.equal(grad, want_grad), tune


@pytest.mark.parametrize("kind,cyclic,n,m,pad", [("tri", False, 1024, 20000, 40), ("penta", True, 256, 5000, 3),
                                               ("tri", True, 64, 33, 7)])
def test_adjoint_band_grad_strided(kind, cyclic, n, m, pad):
    """Batches with a leading dimension above m (g, lam and every state of
    traj n * ld apart): the same results as the contiguous batch, bitwise,
    and the columns past m untouched."""
    say("adjoint + band grad strided", kind, cyclic, n, m, pad)
    f, _ = _factor(kind, cyclic, n)
    steps = 3
    ld = m + pad
    g = inputs.uniform_batch(n, m, seed=60)
    us = [inputs.uniform_batch(n, m, seed=61 + t) for t in range(steps)]
    lam_c, grad_c = f.adjoint_band_grad(dev(g), torch.stack([dev(u) for u in us]))
    gs = torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda")
    gs[:, :m] = dev(g)
    ts = torch.full((steps, n, ld), 7.0, dtype=torch.float64, device="cuda")
    for t in range(steps):
        ts[t, :, :m] = dev(us[t])
    lam_s, grad_s = f.adjoint_band_grad(gs[:, :m], ts[:, :, :m])
    assert lam_s.stride(0) == ld
    assert torch.equal(lam_s, lam_c) and torch.equal(grad_s, grad_c)
    assert torch.all(gs[:, m:] == 7.0) and torch.all(ts[:, :, m:] == 7.0)
