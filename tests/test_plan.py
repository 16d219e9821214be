"""Host logic of the decomposition (no GPU): bb_plan reports the chunk
length, lanes per system, waves per group and coefficient source a call
with m systems takes -- the rules the kernels' measurements chose."""
import ctypes

import numpy as np
import pytest

from paper_2107_05395_amd import _lib, inputs


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def _factor(L, kind, n):
    h = ctypes.c_void_p()
    if kind == "tri":
        bands = inputs.diffusion_tri_bands(n, 1.0)
    elif kind == "tri_cyclic":
        bands, _ = inputs.cn_diffusion_problem(n, 1.0)
    elif kind == "penta":
        bands = inputs.hyperdiffusion_penta_bands(n, 0.25)
    else:
        bands = inputs.ch_penta_bands(n, 0.3)
    arrs = [np.ascontiguousarray(b, dtype=np.float64) for b in bands]
    assert getattr(L, "bb_factor_shared_" + kind)(*(_lib.dptr(a) for a in arrs), n,
                                                  ctypes.byref(h)) == 0
    return h


def plan(L, h, m, what=0, prec=0):
    out = [ctypes.c_int32() for _ in range(4)]
    assert L.bb_plan(h, m, what, prec, *(ctypes.byref(o) for o in out)) == 0
    return tuple(o.value for o in out)


# (kind, n, m, what, precision) -> (chunk, lanes, waves, scalar)
CASES = [
    # large solves: 64 rows, groups of 4 waves at 8 chunks, 8 waves from 16
    ("tri", 512, 1 << 20, 0, 0, (64, 8, 4, 0)),
    ("tri", 256, 1 << 20, 0, 0, (64, 4, 1, 0)),
    ("penta", 1024, 1 << 18, 0, 0, (64, 16, 8, 0)),
    ("tri", 2048, 1 << 16, 0, 0, (64, 32, 8, 0)),
    # refinement: groups of P/4 waves; FP32 right-hand sides: 4 waves from P = 4
    ("tri", 512, 1 << 20, 0, 1, (64, 8, 2, 0)),
    ("tri", 512, 1 << 20, 0, 3, (64, 8, 4, 0)),
    # small batches (fewer than 2^16 lanes of 64-row chunks): shorter chunks
    ("tri", 256, 1024, 0, 0, (32, 8, 1, 0)),
    ("tri", 64, 4096, 0, 0, (16, 4, 1, 0)),
    ("tri", 1024, 64, 0, 0, (32, 32, 1, 0)),
    ("tri", 2048, 256, 0, 0, (64, 32, 8, 0)),        # 32 rows would need 64 chunks
    # fused steppers
    ("penta_cyclic", 256, 1 << 20, 1, 0, (64, 4, 4, 1)),   # one chunk per wave, scalar
    ("penta_cyclic", 512, 70000, 1, 0, (64, 8, 8, 1)),
    ("penta_cyclic", 1024, 1 << 16, 1, 0, (64, 16, 8, 0)),  # LDS table, 8-wave groups
    ("tri_cyclic", 64, 1 << 16, 1, 0, (32, 2, 2, 1)),      # below two waves per SIMD
    ("tri_cyclic", 128, 1 << 15, 1, 0, (32, 4, 4, 1)),
    ("tri_cyclic", 64, 4096, 1, 0, (16, 4, 4, 1)),         # small batch, still scalar
    ("tri_cyclic", 1024, 64, 1, 0, (32, 32, 8, 0)),
    ("penta_cyclic", 300, 100, 1, 0, (32, 16, 1, 0)),      # ragged: one wave per group
]


@pytest.mark.parametrize("kind,n,m,what,prec,want", CASES)
def test_plan_rules(L, kind, n, m, what, prec, want):
    h = _factor(L, kind, n)
    assert plan(L, h, m, what, prec) == want
    L.bb_factor_destroy(h)


def test_plan_follows_tuning_variables(L, tuning):
    h = _factor(L, "penta_cyclic", 256)
    tuning.set("max_chunk", "32")
    assert plan(L, h, 1 << 20, 0, 0)[:2] == (32, 8)
    tuning.set("max_chunk", None)
    tuning.set("ch_uniform", "0")
    assert plan(L, h, 1 << 20, 1, 0) == (64, 4, 1, 0)
    tuning.set("waves_per_system", "2")
    assert plan(L, h, 1 << 20, 1, 0) == (64, 4, 2, 0)
    L.bb_factor_destroy(h)


def test_plan_argument_errors(L):
    h = _factor(L, "tri", 64)
    out = ctypes.c_int32()
    assert L.bb_plan(None, 10, 0, 0, ctypes.byref(out), None, None, None) == -1
    assert L.bb_plan(h, 0, 0, 0, ctypes.byref(out), None, None, None) == -1
    assert L.bb_plan(h, 10, 2, 0, ctypes.byref(out), None, None, None) == -1
    assert L.bb_plan(h, 10, 0, 9, ctypes.byref(out), None, None, None) == -1
    assert L.bb_plan(h, 10, 0, 0, None, None, None, None) == 0
    L.bb_factor_destroy(h)


def test_empty_batch_pads_rows_at_64k_strides():
    """empty_batch: an (n, m) view with ld = m + 32 where the row's byte
    stride is a multiple of 64 KiB, ld = m otherwise, or the padding asked for."""
    import torch
    from paper_2107_05395_amd import empty_batch
    t = empty_batch(8, 1 << 18, device="cpu")
    assert t.shape == (8, 1 << 18) and t.stride() == ((1 << 18) + 32, 1)
    assert empty_batch(8, 1000, device="cpu").stride() == (1000, 1)
    assert empty_batch(8, 8192, dtype=torch.float32, device="cpu").stride() == (8192, 1)
    assert empty_batch(8, 16384, dtype=torch.float32, device="cpu").stride() == (16384 + 32, 1)
    assert empty_batch(8, 100, device="cpu", pad=7).stride() == (107, 1)
