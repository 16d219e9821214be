"""Helpers shared by the GPU tests (device transfer, error metrics)."""
import numpy as np
import torch


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def rel_err(x, ref, axis=0):
    """Max over systems of the per-system relative 2-norm error."""
    x, ref = np.asarray(x, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    num = np.linalg.norm(x - ref, axis=axis)
    den = np.linalg.norm(ref, axis=axis)
    return float(np.max(num / np.where(den == 0, 1.0, den)))


def say(*args):
    print(*args, flush=True)


def fp64_tol(kappa=1.0, steps=1):
    """Tolerance of an FP64 comparison between two correct implementations.

    1e-12 is the bar.  An LU solve without pivoting is backward stable, so its
    computed solution carries a forward error of up to about kappa(A) * u
    (u = 2^-53) on top of the input's; two implementations that round in
    different orders (the chunked sweeps and the oracle's sequential loops)
    can therefore differ by up to about 2 kappa u per solve, compounded over
    `steps` implicit steps whose amplification stays near 1.  Measured: the
    oracle against an FFT solve of the periodic Cahn-Hilliard matrix differs
    by 0.24 kappa u at n = 256, 512 and 1024.  The bar is widened only where
    2 steps kappa u exceeds it (kappa above about 4500 per step)."""
    return max(1e-12, 2.0 * steps * kappa * 2.0 ** -53)


def lbar_tol(kappa, steps, c0, ref_lbar):
    """Tolerance for the relative error of lbar - 1, lbar the ensemble mean of
    l = 1 / (1 - <C^2>) over the m runs of c0.

    States: lbar - 1 is about <C^2>, and an error dC of the states moves
    <C^2> by about 2 |C| |dC|, so the relative error of lbar - 1 is about
    2 |dC| / rms(C).  The state error is bounded at the scale of the start,
    fp64_tol(kappa, steps) max|C_0| (the rounding of the explicit right-hand
    side reaches the low modes, which the solve passes undamped), while
    rms(C) shrinks as the hyperdiffusion smooths the start; <C^2> = 1 - 1/lbar
    is read from the oracle's lbar.
    Mean: the oracle averages the l of m runs pairwise, an absolute error of
    up to about log2(m) u lbar, which is relative to lbar - 1."""
    u = 2.0 ** -53
    ref = np.asarray(ref_lbar, dtype=np.float64)
    c2 = 1.0 - 1.0 / ref
    m = np.asarray(c0).shape[1]
    states = 2.0 * fp64_tol(kappa, steps) * float(np.max(np.abs(c0))) / float(np.sqrt(np.min(c2)))
    mean = 4.0 * max(1.0, np.log2(m)) * u * float(np.max(ref)) / float(np.min(ref - 1.0))
    return states + mean
