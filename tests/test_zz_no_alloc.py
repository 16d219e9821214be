"""The allocation-free band gradient (bb_band_grad_noalloc, partial sums in
the library's own device array) against bb_band_grad (caller workspace),
through the C ABI: two calls in a row, the second on a smaller input, each
to the FP64 bar, on top of a non-zero gradient (+=)."""
import numpy as np
import pytest
import torch

from paper_2107_05395_amd import Factor, _lib, inputs
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _case(kind, n, m, seed):
    g = inputs.rng(seed)
    if kind == "tri":
        D = g.uniform(0.5, 1.5, n)
        f = Factor.tri(-0.5 * D, 1.0 + D, -0.5 * D)
    else:
        f = Factor.penta(*inputs.hyperdiffusion_penta_bands(n, 0.25), cyclic=True)
    lam = dev(g.uniform(-1, 1, (n, m)))
    x = dev(g.uniform(-1, 1, (n, m)))
    start = g.uniform(-1, 1, (f.nbands, n))
    return f, lam, x, start


def _both(f, lam, x, start):
    want = f.band_grad(lam, x, grad=dev(start))
    got = f.band_grad_noalloc(lam, x, dev(start))
    return host(got), host(want)


def test_scratch_size_is_declared():
    assert _lib.lib().bb_band_grad_scratch_bytes() == 4 << 20


@pytest.mark.parametrize("first,second", [
    (("penta", 1024, 70000), ("tri", 256, 3000)),
    (("tri", 1024, (1 << 16) + 7), ("tri", 512, 100)),
])
def test_noalloc_band_grad_matches_workspace_entry_point(first, second):
    for i, (kind, n, m) in enumerate((first, second)):
        say("noalloc band grad", kind, n, m)
        f, lam, x, start = _case(kind, n, m, seed=7 + i + n)
        got, want = _both(f, lam, x, start)
        scale = np.max(np.abs(want - start), axis=1, keepdims=True)
        err = float(np.max(np.abs(got - want) / scale))
        say("  err", err)
        assert err < 1e-12
        # the array keeps the last call's contents: a repeat gives the same bits
        again = host(f.band_grad_noalloc(lam, x, dev(start)))
        assert np.array_equal(again, got)
