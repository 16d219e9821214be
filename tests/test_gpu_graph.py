"""The C-ABI entry points enqueue kernels only (no allocation, no memset, no
host synchronisation once a call's coefficient table exists), so a sequence
of solves and fused steps can be captured in a HIP graph and replayed.  Each
replay must reproduce the eager results bitwise, with eager work and
synchronisations between the replays."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2107_05395_amd import inputs
from tests.gpu_util import dev, host, rel_err, say

pytestmark = pytest.mark.gpu


def test_solves_and_steps_replay_in_a_graph():
    from paper_2107_05395_amd import Factor
    n, m = 512, 3000
    tri = Factor.tri(*inputs.diffusion_tri_bands(n, 1.0))
    pb, pw = inputs.cn_hyperdiffusion_problem(n, 0.8)
    penta = Factor.penta(*pb, cyclic=True)
    ch = Factor.cahn_hilliard(n, 2 * math.pi, 0.01, 1e-3)
    rhs_h = inputs.uniform_batch(n, m, seed=81)
    rhs = dev(rhs_h)
    c0 = dev(inputs.uniform_batch(n, m, seed=82, lo=-0.1, hi=0.1))
    outs = [torch.empty_like(rhs) for _ in range(5)]

    def work():
        tri.solve(rhs, out=outs[0])
        tri.solve(rhs, out=outs[1], precision="f32r")
        penta.solve(rhs, out=outs[2])
        penta.cn_step(rhs, pw, steps=5, out=outs[3])
        ch.ch_step(c0, ch.alpha, steps=3, out=outs[4])

    work()                                     # eager: builds and uploads every table
    torch.cuda.synchronize()
    eager = [host(o) for o in outs]
    assert rel_err(eager[0], oracle.tri_solve(*inputs.diffusion_tri_bands(n, 1.0), rhs_h)) < 1e-12
    assert rel_err(eager[3], oracle.cn_step(pb, pw, rhs_h, steps=5)) < 1e-12

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            work()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        tri.solve(c0, out=torch.empty_like(c0))   # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert np.array_equal(host(o), eager[i]), (rep, i)
        say("graph replay", rep, "ok")


def test_fused_backward_replays_in_a_graph():
    """bb_adjoint_band_grad on the fused kernel and on the step-by-step path
    (an odd number of steps: the last adjoint is copied out of the
    workspace), captured once and replayed: every replay gives the eager
    adjoints and band gradients bitwise."""
    import ctypes
    from paper_2107_05395_amd import Factor, _lib
    from paper_2107_05395_amd.solver import check
    L = _lib.lib()
    cases = []
    for kind, n, m, steps in (("tri", 1024, 20000, 2), ("tri", 64, 33, 3)):
        f = Factor.tri(*inputs.random_dominant_tri(n, seed=n))
        g = dev(inputs.uniform_batch(n, m, seed=90))
        traj = torch.stack([dev(inputs.uniform_batch(n, m, seed=91 + t)) for t in range(steps)])
        lam = torch.empty_like(g)
        grad = torch.zeros(3, n, dtype=torch.float64, device="cuda")
        nbytes = L.bb_adjoint_band_grad_workspace_bytes(f.handle, m, m)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        cases.append((f, g, traj, lam, grad, ws, n, m, steps))
    assert cases[0][0].adjoint_band_grad_fused(20000) and not cases[1][0].adjoint_band_grad_fused(33)

    def work(stream):
        for f, g, traj, lam, grad, ws, n, m, steps in cases:
            check(L.bb_adjoint_band_grad(f.handle, ctypes.c_void_p(g.data_ptr()),
                                         ctypes.c_void_p(traj.data_ptr()),
                                         ctypes.c_void_p(lam.data_ptr()), m, m, steps,
                                         ctypes.c_void_p(grad.data_ptr()),
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), stream))

    work(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))   # eager: tables uploaded
    torch.cuda.synchronize()
    eager = [(host(c[3]), host(c[4])) for c in cases]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            work(ctypes.c_void_p(side.cuda_stream))
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for c in cases:
            c[3].fill_(float("nan"))
            c[4].zero_()
        cases[0][0].solve(cases[0][1], out=torch.empty_like(cases[0][1]))   # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, c in enumerate(cases):
            assert np.array_equal(host(c[3]), eager[i][0]), (rep, i)
            assert np.array_equal(host(c[4]), eager[i][1]), (rep, i)
