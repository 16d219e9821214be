"""GPU parity at the full sizes of the configured workloads, in the launch
configuration bench.py times (same library calls, same chunking), on sampled
systems the oracle solves one by one, plus properties that hold at any size.

  * diffusion n=256, m=1024: every system.
  * diffusion n=512, m=2^20: FP64, FP32+refine and FP32 right-hand sides with
    refinement, 512 sampled systems.
  * hyperdiffusion n=1024, m=2^18 (sine-mode RHS): the same three forms, sampled.
  * Cahn-Hilliard n=256, m=2^20: 10 fused steps, sampled systems; mass of
    every system conserved.
  * differentiated diffusion n=1024, m=2^16, T=100, checkpoint every 10:
    dL/du0 on sampled systems; dL/dD at full size with every system but a
    sampled set zeroed (the zero systems contribute exactly nothing, so the
    full launch must equal the oracle's sum over the sample, scaled by
    |sample|/m); and a central finite-difference check of dL/dD on the
    full random batch.
  * Crank-Nicolson grid, largest point (n=1024, m=2^16, periodic tri and
    penta, 1000 steps): the fused launch and 1000 single-step launches,
    sampled systems.
  * Cahn-Hilliard coarsening, L = 2 pi (n=256, m=2^20, dt = 0.1 dx): the
    statistic after each of 4 steps over all 2^20 runs against the oracle.
  * forced Cahn-Hilliard flow-pattern batch (768 x 768 runs, n=512): 20
    steps, sampled runs.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2107_05395_amd import inputs
from tests.gpu_util import fp64_tol, lbar_tol, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    from paper_2107_05395_amd import solver  # noqa: F401
    oracle.build()


def sample_cols(m, count=512, seed=0):
    g = np.random.default_rng(seed)
    return np.unique(np.r_[0, m - 1, g.choice(m, size=min(count, m), replace=False)])


def cols_of(t, cols):
    return t[:, torch.from_numpy(cols).to(t.device)].cpu().numpy()


def test_diffusion_n256_m1024_every_system():
    from paper_2107_05395_amd import Factor
    spec = inputs.WORKLOADS["diffusion_n256_m1024"]
    n, m = spec["n"], spec["m"]
    bands = inputs.diffusion_tri_bands(n, spec["r"])
    rhs = inputs.uniform_batch(n, m, seed=spec["seed"])
    f = Factor.tri(*bands)
    ref = oracle.tri_solve(*bands, rhs)
    t = torch.from_numpy(rhs).cuda()
    assert rel_err(f.solve(t).cpu().numpy(), ref) < 1e-12
    assert rel_err(f.solve(t, precision="f32r").cpu().numpy(), ref) < 1e-10


def test_diffusion_n512_m2p20_sampled():
    from paper_2107_05395_amd import Factor
    spec = inputs.WORKLOADS["diffusion_n512_m1048576"]
    n, m = spec["n"], spec["m"]
    say("generating", n, m)
    bands = inputs.diffusion_tri_bands(n, spec["r"])
    rhs = inputs.uniform_batch(n, m, seed=spec["seed"])
    f = Factor.tri(*bands)
    t = torch.from_numpy(rhs).cuda()
    cols = sample_cols(m)
    ref = oracle.tri_solve(*bands, rhs[:, cols])
    x = torch.empty_like(t)
    for prec, tol in (("f64", 1e-12), ("f32r", 1e-10)):
        f.solve(t, out=x, precision=prec)
        err = rel_err(cols_of(x, cols), ref)
        say(prec, "max rel err", err)
        assert err < tol
    # the paper's mapping on the same input
    f.solve_thread_per_system(t, out=x)
    assert rel_err(cols_of(x, cols), ref) < 1e-12
    # FP32 right-hand-side data (the same draws rounded), refined to double
    t32 = t.float()
    ref32 = oracle.tri_solve(*bands, rhs[:, cols].astype(np.float32).astype(np.float64))
    f.solve(t32, out=x, precision="f32rhs")
    assert rel_err(cols_of(x, cols), ref32) < 1e-10


def test_hyperdiffusion_n1024_m2p18_sampled():
    from paper_2107_05395_amd import Factor
    spec = inputs.WORKLOADS["hyperdiffusion_n1024_m262144"]
    n, m = spec["n"], spec["m"]
    bands = inputs.hyperdiffusion_penta_bands(n, spec["r"])
    rhs = inputs.sine_mode_batch(n, m, seed=spec["seed"])
    f = Factor.penta(*bands)
    t = torch.from_numpy(rhs).cuda()
    cols = sample_cols(m)
    ref = oracle.penta_solve(*bands, rhs[:, cols])
    x = torch.empty_like(t)
    for prec, tol in (("f64", 1e-12), ("f32r", 1e-10)):
        f.solve(t, out=x, precision=prec)
        err = rel_err(cols_of(x, cols), ref)
        say(prec, "max rel err", err)
        assert err < tol
    t32 = t.float()
    ref32 = oracle.penta_solve(*bands, rhs[:, cols].astype(np.float32).astype(np.float64))
    f.solve(t32, out=x, precision="f32rhs")
    assert rel_err(cols_of(x, cols), ref32) < 1e-10


def test_cahn_hilliard_n256_m2p20_sampled():
    from paper_2107_05395_amd import Factor
    spec = inputs.WORKLOADS["cahn_hilliard_n256_m1048576"]
    n, m = spec["n"], spec["m"]
    sigma, alpha = oracle.ch_coefficients(spec["gamma"], 2 * math.pi / n, spec["dt"])
    c0 = inputs.uniform_batch(n, m, seed=spec["seed"], lo=-0.1, hi=0.1)
    f = Factor.cahn_hilliard(n, 2 * math.pi, spec["gamma"], spec["dt"])
    t = torch.from_numpy(c0).cuda()
    steps = 10
    out = f.ch_step(t, f.alpha, steps=steps)
    cols = sample_cols(m, 256)
    ref = oracle.ch_step(c0[:, cols], sigma, alpha, steps=steps)
    err = rel_err(cols_of(out, cols), ref)
    say("CH 10 steps max rel err", err)
    assert err < 1e-12
    # mass of every system: rounding bound from the right-hand side magnitude
    # |f| <= |C| (1 + 4 alpha) of each step (as in test_gpu_grad_ch)
    drift = (out.sum(dim=0) - t.sum(dim=0)).abs().max().item()
    cmax = max(out.abs().max().item(), t.abs().max().item())
    assert drift < 4 * steps * n * np.finfo(float).eps * cmax * (1 + 4 * alpha)


def test_differentiated_diffusion_n1024_m2p16():
    from paper_2107_05395_amd import banded_rollout, mse_loss
    spec = inputs.WORKLOADS["adjoint_diffusion_n1024_m65536"]
    n, m, r, T, every = spec["n"], spec["m"], spec["r"], spec["steps"], spec["checkpoint"]
    g = inputs.rng(spec["seed"])
    D0 = g.uniform(0.5, 1.5, n)
    u0 = inputs.uniform_batch(n, m, seed=spec["seed"] + 1)
    y = inputs.uniform_batch(n, m, seed=spec["seed"] + 2)
    tu0_host, ty = torch.from_numpy(u0).cuda(), torch.from_numpy(y).cuda()

    def run(D_np, prec, grad=True):
        D = torch.tensor(D_np, requires_grad=grad)
        tu = tu0_host.clone().requires_grad_(grad)
        uT = banded_rollout(tu, (-r * D, 1 + 2 * r * D, -r * D), steps=T, checkpoint_every=every,
                            precision=prec)
        loss = mse_loss(uT, ty)
        if grad:
            loss.backward()
            return loss.item(), D.grad.numpy(), tu.grad, uT.detach()
        return loss.item()

    cols = sample_cols(m, 256)
    scale = len(cols) / m
    # (1) every system zero except the sample
    u0_s, y_s = np.zeros_like(u0), np.zeros_like(y)
    u0_s[:, cols], y_s[:, cols] = u0[:, cols], y[:, cols]
    loss_ref, dD_ref, du0_ref = oracle.diffusion_loss_and_grads(D0, r, u0[:, cols], y[:, cols], T)
    tu0_host.copy_(torch.from_numpy(u0_s))
    ty.copy_(torch.from_numpy(y_s))
    for prec, tol in (("f64", 1e-12), ("f32r", 1e-10)):
        loss, dD, du0, _ = run(D0, prec)
        say(prec, "loss", loss, loss_ref * scale)
        assert abs(loss - loss_ref * scale) < tol * loss_ref * scale
        assert np.max(np.abs(dD - dD_ref * scale)) < tol * np.max(np.abs(dD_ref * scale))
        assert rel_err(cols_of(du0, cols), du0_ref * scale) < tol
    # (2) the full random batch: per-system gradients on the sample, and
    #     central differences of the loss along random directions
    tu0_host.copy_(torch.from_numpy(u0))
    ty.copy_(torch.from_numpy(y))
    loss, dD, du0, _ = run(D0, "f64")
    # per-system gradients do not depend on the other systems
    assert rel_err(cols_of(du0, cols), du0_ref * scale) < 1e-12
    rng = np.random.default_rng(7)
    h = 1e-5
    for _ in range(2):
        v = rng.standard_normal(n)
        fd = (run(D0 + h * v, "f64", False) - run(D0 - h * v, "f64", False)) / (2 * h)
        say("fd", fd, dD @ v)
        assert abs(fd - dD @ v) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("workload", ["cn_diffusion_grid", "cn_hyperdiffusion_grid"])
def test_crank_nicolson_grid_largest_point_sampled(workload):
    from paper_2107_05395_amd import Factor
    spec = inputs.WORKLOADS[workload]
    n, m, T, sigma = max(spec["ns"]), max(spec["ms"]), spec["steps"], spec["sigma"]
    diff = spec["problem"] == "diffusion"
    bands, w = (inputs.cn_diffusion_problem if diff else inputs.cn_hyperdiffusion_problem)(n, sigma)
    f = Factor.tri(*bands, cyclic=True) if diff else Factor.penta(*bands, cyclic=True)
    c0 = inputs.uniform_batch(n, m, seed=spec["seed"] + n + m)
    cols = sample_cols(m, 64, seed=5)
    ref = oracle.cn_step(bands, w, c0[:, cols], steps=T)
    t = torch.from_numpy(c0).cuda()
    fused = f.cn_step(t, w, steps=T)
    err = rel_err(cols_of(fused, cols), ref)
    a, b = t.clone(), torch.empty_like(t)
    for _ in range(T):
        f.cn_step(a, w, out=b)
        a, b = b, a
    err1 = rel_err(cols_of(a, cols), ref)
    say(workload, "fused", err, "per step", err1)
    # after 1000 steps the states have decayed to near their means while the
    # rounding accumulated at the scale of the start: bound by the start
    assert np.max(np.abs(cols_of(fused, cols) - ref)) < 1e-12 * T ** 0.5 * np.max(np.abs(c0[:, cols]))
    assert np.max(np.abs(cols_of(a, cols) - ref)) < 1e-12 * T ** 0.5 * np.max(np.abs(c0[:, cols]))


def test_ch_coarsening_statistic_full_batch():
    from paper_2107_05395_amd import Factor
    spec = inputs.WORKLOADS["ch_coarsening_L2pi"]
    n, m, L, gamma = spec["n"], spec["m"], spec["length"], spec["gamma"]
    dt = 0.1 * L / n
    sigma, alpha = oracle.ch_coefficients(gamma, L / n, dt)
    f = Factor.cahn_hilliard(n, L, gamma, dt)
    c0 = inputs.uniform_batch(n, m, seed=spec["seed"], lo=-0.1, hi=0.1)
    steps = 4
    ref, ref_c = oracle.ch_coarsening(c0, sigma, alpha, steps, 1)
    out, lbar = f.ch_step_stats(torch.from_numpy(c0).cuda(), f.alpha, steps=steps, every=1)
    lb = lbar.cpu().numpy()
    err = float(np.max(np.abs(lb - ref) / (ref - 1.0)))
    tol = lbar_tol(1.0 + 16.0 * sigma, steps, c0, ref)
    say("coarsening full batch lbar", lb, "rel err of lbar - 1", err, "tol", tol)
    assert err < tol
    cols = sample_cols(m, 512, seed=6)
    assert rel_err(cols_of(out, cols), ref_c[:, cols]) < 1e-12


def test_forced_flowmap_batch_sampled():
    """The forced flow-pattern batch at its full size (768 x 768 runs, n = 512)
    in the bench's launch configuration, 20 steps, sampled runs."""
    import math
    from paper_2107_05395_amd import Factor
    spec = inputs.WORKLOADS["ch_forced_flowmap_v05"]
    n, L, G = spec["n"], spec["length"], spec["grid"]
    m = G * G
    dx = L / n
    dt = 0.1 * dx
    sigma, alpha = oracle.ch_coefficients(spec["gamma"], dx, dt)
    f0 = np.repeat(np.linspace(spec["f0"][0], spec["f0"][1], G), G)
    mean = np.tile(np.linspace(spec["mean"][0], spec["mean"][1], G), G)
    v, k = np.full(m, spec["v"]), np.full(m, spec["k"])
    beta, amp, kdx = oracle.ch_forced_parameters(dt, dx, v, f0, k)
    c0 = mean + inputs.uniform_batch(n, m, seed=spec["seed"], lo=-0.1, hi=0.1)
    cols = sample_cols(m, 256, seed=7)
    ref = oracle.ch_forced_step(c0[:, cols], sigma, alpha, beta[cols], amp[cols], kdx[cols],
                                steps=20)
    f = Factor.cahn_hilliard(n, L, spec["gamma"], dt)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = f.ch_forced_step(dv(c0), dt, dx, dv(v), dv(f0), dv(k), steps=20)
    err = rel_err(cols_of(out, cols), ref)
    tol = fp64_tol(1.0 + 16.0 * sigma, 20)
    say("forced flow-map batch, 20 steps, rel err", err, "tol", tol)
    assert err < tol
