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
