"""Differentiable batched solves.

The backward pass of x = A^{-1} b is one transposed solve with the same
shared factor, lam = A^{-T} dL/dx (so dL/db = lam), plus the band gradients
dL/dA_ij = -sum_k lam_i x_j reduced over the batch into the shared bands.
Both run in libbandbatch's kernels; torch only sees the results.

``banded_rollout`` differentiates T implicit steps u_t = A^{-1} u_{t-1}
with activation checkpointing: the forward pass keeps every
``checkpoint_every``-th state, and the backward pass recomputes each segment
from its checkpoint before walking it backwards.  In FP64 the steps run in
the fused time-stepping kernel with the identity as right-hand-side
stencil: the forward pass takes one launch per segment with the state held
on chip, and the recomputation of a segment one launch of the same kernel
that also stores every intermediate state.  A fused launch of k steps, a
trajectory launch and k single-step launches agree bitwise (same kernel
arithmetic and decomposition), so the recomputed states equal the forward's.
The adjoint recursion lam_t = A^{-T} lam_{t+1} is stepped the same way,
one launch per segment on the factor's transposed solve, and the same launch
reduces each adjoint against its recomputed state into the band gradients
(bb_adjoint_band_grad): no adjoint state is written to memory.
"""
from __future__ import annotations

import torch

from .solver import Factor, mse_loss_grad


def _host_bands(bands):
    return [b.detach().to("cpu", torch.float64).numpy() for b in bands]


def _factor_from(bands, kind: str, cyclic: bool) -> Factor:
    host = _host_bands(bands)
    return Factor.tri(*host, cyclic=cyclic) if kind == "tri" else Factor.penta(*host, cyclic=cyclic)


_SIDE_STREAMS: dict = {}


def _side_stream(device, which: int) -> "torch.cuda.Stream":
    """Extra streams per device (default priority) for work that may overlap
    the main chain of solves."""
    key = (torch.device(device).index, which)
    if key not in _SIDE_STREAMS:
        _SIDE_STREAMS[key] = torch.cuda.Stream(device=device)
    return _SIDE_STREAMS[key]


def _kind(nb: int) -> str:
    if nb not in (3, 5):
        raise ValueError("need 3 (tri) or 5 (penta) bands")
    return "tri" if nb == 3 else "penta"


class BandedSolve(torch.autograd.Function):
    """x = A(bands)^{-1} rhs, differentiable in rhs and in every band."""

    @staticmethod
    def forward(ctx, rhs, cyclic, precision, *bands):
        f = _factor_from(bands, _kind(len(bands)), cyclic)
        x = f.solve(rhs.contiguous(), precision=precision)
        ctx.factor, ctx.precision = f, precision
        ctx.band_devices = [b.device for b in bands]
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        f = ctx.factor
        lam = f.adjoint(gx.contiguous(), precision=ctx.precision)
        gb = f.band_grad(lam, x)
        return (lam, None, None, *[gb[q].to(d) for q, d in enumerate(ctx.band_devices)])


def banded_solve(rhs, bands, cyclic: bool = False, precision: str = "f64"):
    return BandedSolve.apply(rhs, cyclic, precision, *bands)


def _identity(f: Factor):
    w = [0.0] * f.nbands
    w[f.nbands // 2] = 1.0
    return w


def _trajectory(f: Factor, u, k: int, precision: str):
    """[u_{t+1}, ..., u_{t+k}] from u_t."""
    if precision == "f64":
        return list(f.cn_trajectory(u, _identity(f), k).unbind(0))
    out = []
    for _ in range(k):
        u = f.solve(u, precision=precision)
        out.append(u)
    return out


def _advance(f: Factor, u, k: int, precision: str):
    """u_{t+k} from u_t: k solves u' = A^{-1} u.  FP64 runs them in one launch
    of the fused stepper (A u' = I u), or for long systems as k single steps
    of the same form (the steps the backward trajectory recomputes); other
    precisions solve step by step."""
    if precision == "f64" and f.long:
        for _ in range(k):
            u = f.cn_step(u, _identity(f), steps=1)
        return u
    if precision == "f64":
        return f.cn_step(u, _identity(f), steps=k)
    for _ in range(k):
        u = f.solve(u, precision=precision)
    return u


class BandedRollout(torch.autograd.Function):
    """u_T after `steps` solves u_t = A(bands)^{-1} u_{t-1}, checkpointed;
    A periodic (corner entries from the bands, Section 3.3) when cyclic."""

    @staticmethod
    def forward(ctx, u0, steps, checkpoint_every, precision, cyclic, *bands):
        if steps < 1 or checkpoint_every < 1:
            raise ValueError("steps and checkpoint_every must be >= 1")
        f = _factor_from(bands, _kind(len(bands)), bool(cyclic))
        u = u0.detach().contiguous()
        checkpoints = [u]
        t = 0
        while t < steps:
            k = min(checkpoint_every, steps - t)
            u = _advance(f, u, k, precision)
            t += k
            if t < steps:
                checkpoints.append(u)
        ctx.factor, ctx.steps, ctx.every, ctx.precision = f, steps, checkpoint_every, precision
        ctx.band_devices = [b.device for b in bands]
        ctx.checkpoints = checkpoints
        return u

    @staticmethod
    def backward(ctx, g_out):
        f, steps, every, prec = ctx.factor, ctx.steps, ctx.every, ctx.precision
        g = g_out.contiguous()
        main = torch.cuda.current_stream(g.device)
        # The states of the next segment (walking backwards) depend only on
        # its checkpoint: they are recomputed on a second stream while the
        # current segment's adjoints run.  Outside FP64 the band-gradient
        # reductions, which depend only on lam_t and u_t and not on the next
        # adjoint solve, run on a third stream beside the chain of solves;
        # their order among themselves, and so the sums, stay fixed.  All
        # streams default priority.
        side = _side_stream(g.device, 0)
        ahead = _side_stream(g.device, 1)
        side.wait_stream(main)
        ahead.wait_stream(main)
        gb = torch.zeros(f.nbands, f.n, dtype=torch.float64, device=g.device)
        gb.record_stream(side)

        # FP64: the adjoints of a segment and their band gradients in one
        # call (bb_adjoint_band_grad: transposed solves with the factor's own
        # A^T = U^T L^T, reduced against the recomputed states as they go)
        traj = prec == "f64"

        def recompute(i):
            # states of segment i from checkpoint i, on `ahead`: FP64 the
            # (k, n, m) trajectory u_{s+1} .. u_e, else the list u_s .. u_e
            s = i * every
            k = min(s + every, steps) - s
            with torch.cuda.stream(ahead):
                if traj:
                    return f.cn_trajectory(ctx.checkpoints[i], _identity(f), k)
                return [ctx.checkpoints[i]] + _trajectory(f, ctx.checkpoints[i], k, prec)

        # segments [s, e): states u_s .. u_e; checkpoint i holds u_{i*every}
        last = len(ctx.checkpoints) - 1
        pending = recompute(last)
        for i in reversed(range(last + 1)):
            s = i * every
            e = min(s + every, steps)
            main.wait_stream(ahead)                 # this segment's states are ready
            states = pending
            if traj:
                states.record_stream(main)
            else:
                for u in states:
                    u.record_stream(main)
            pending = recompute(i - 1) if i > 0 else None
            if traj:
                # d_{t-1} = A^{-T} d_t for t = e .. s+1 from d_e = g, with
                # gb += -sum_t d_{t-1} u_t^T over the segment
                g, _ = f.adjoint_band_grad(g, states, gb)
                del states
                continue
            for t in range(e, s, -1):          # u_t = A^{-1} u_{t-1}
                lam = f.adjoint(g, precision=prec)
                side.wait_stream(main)
                with torch.cuda.stream(side):
                    f.band_grad(lam, states[t - s], gb)
                lam.record_stream(side)
                states[t - s].record_stream(side)
                g = lam
            del states
        main.wait_stream(side)
        ctx.checkpoints = None
        return (g, None, None, None, None,
                *[gb[q].to(d) for q, d in enumerate(ctx.band_devices)])


def banded_rollout(u0, bands, steps: int, checkpoint_every: int = 10, precision: str = "f64",
                   cyclic: bool = False):
    return BandedRollout.apply(u0, steps, checkpoint_every, precision, cyclic, *bands)


class MSELoss(torch.autograd.Function):
    """mean((u - target)^2) over every entry, gradient from the same kernel."""

    @staticmethod
    def forward(ctx, u, target):
        loss, grad = mse_loss_grad(u.contiguous(), target.contiguous())
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, gl):
        (grad,) = ctx.saved_tensors
        return grad * gl, None


def mse_loss(u, target):
    return MSELoss.apply(u, target)
