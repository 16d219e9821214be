"""CPU-only checks of the C ABI: the library loads, exports every function
include/bandbatch.h declares, and its host-side validation (factorisation,
pivots, capacitance, argument checks, error strings) behaves as documented.
No call here touches a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2107_05395_amd import _lib, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bandbatch.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2107_05395_amd import build
        build.build(verbose=False)
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bb_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ["bb_factor_shared_tri", "bb_factor_shared_penta", "bb_factor_shared_tri_cyclic",
                 "bb_factor_shared_penta_cyclic", "bb_solve_batch_tri", "bb_solve_batch_penta",
                 "bb_solve_batch_tri_adjoint", "bb_solve_batch_penta_adjoint", "bb_band_grad",
                 "bb_ch_step", "bb_ch_step_stats", "bb_ch_forced_step", "bb_factor_ch", "bb_cn_step",
                 "bb_status_string", "bb_last_error_message"]:
        assert must in names


def test_every_declared_symbol_is_exported(L):
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def _factor(L, kind, bands, n):
    h = ctypes.c_void_p()
    arrs = [np.ascontiguousarray(b, dtype=np.float64) for b in bands]
    st = getattr(L, "bb_factor_shared_" + kind)(*(_lib.dptr(a) for a in arrs), n, ctypes.byref(h))
    return st, h


def test_factor_ok_and_info(L):
    n = 512
    st, h = _factor(L, "tri", inputs.diffusion_tri_bands(n, 1.0), n)
    assert st == 0 and h.value
    nn, kind, chunk = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    assert L.bb_factor_info(h, ctypes.byref(nn), ctypes.byref(kind), ctypes.byref(chunk)) == 0
    assert (nn.value, kind.value) == (n, 0)
    assert chunk.value in (4, 8, 16, 32, 64, 128) and chunk.value * 64 >= n
    assert L.bb_factor_destroy(h) == 0
    assert L.bb_factor_destroy(None) == 0


def test_zero_pivot_rejected(L):
    n = 3
    st, h = _factor(L, "tri", ([0, 1, 1], [0, 1, 1], [1, 1, 0]), n)
    assert st == -2 and not h.value
    assert b"pivot" in L.bb_last_error_message()
    # nonsingular, but the leading 2x2 minor is singular: the method does not pivot
    st, _ = _factor(L, "tri", ([0, 1, 1], [1, 1, 2], [1, 1, 0]), n)
    assert st == -2
    st, _ = _factor(L, "penta", ([0] * 5, [0] * 5, [0, 1, 1, 1, 1], [0] * 5, [0] * 5), 5)
    assert st == -2
    st, _ = _factor(L, "tri", ([0, -1, -1], [1, np.nan, 1], [-1, -1, 0]), n)
    assert st == -2


def test_singular_capacitance_rejected(L):
    # periodic tri with b = a + c everywhere: A has the constant vector in its null space
    n = 6
    st, _ = _factor(L, "tri_cyclic", (np.full(n, -1.0), np.full(n, 2.0), np.full(n, -1.0)), n)
    assert st in (-2, -3)
    assert L.bb_last_error_message()


def test_size_limits(L):
    st, _ = _factor(L, "tri", ([1.0], [2.0], [1.0]), 1)
    assert st == 0
    st, _ = _factor(L, "tri", ([], [], []), 0)
    assert st == -1
    st, _ = _factor(L, "tri_cyclic", ([1.0] * 2, [4.0] * 2, [1.0] * 2), 2)
    assert st == -1
    st, _ = _factor(L, "penta_cyclic", *([[[1.0] * 4] * 5, 4]))
    assert st == -1
    big = L.bb_max_n() + 1
    st, _ = _factor(L, "tri", (np.ones(big), np.full(big, 3.0), np.ones(big)), big)
    assert st == -6
    assert b"bb_max_n" in L.bb_last_error_message()
    st, h = _factor(L, "penta", [np.ones(1024)] * 2 + [np.full(1024, 9.0)] + [np.ones(1024)] * 2, 1024)
    assert st == 0
    L.bb_factor_destroy(h)


def test_long_systems_host_checks(L):
    """Above tri n = 2048 / penta n = 1024 the solves take the three-launch
    long-system path: FP64 only, out of place; the fused steppers are not
    built for it and the (forced) Cahn-Hilliard step takes one out-of-place
    step per call.  All of it is checked on the host, before any device call."""
    fake = ctypes.c_void_p(0x1000)
    other = ctypes.c_void_p(0x2000)
    n = 1025
    st, hp = _factor(L, "penta", [np.ones(n)] * 2 + [np.full(n, 9.0)] + [np.ones(n)] * 2, n)
    assert st == 0
    chunk, lanes, waves, scalar = (ctypes.c_int32() for _ in range(4))
    assert L.bb_plan(hp, 100000, 0, 0, ctypes.byref(chunk), ctypes.byref(lanes), ctypes.byref(waves),
                     ctypes.byref(scalar)) == 0
    assert chunk.value == 64 and lanes.value == 17 and waves.value == 1 and scalar.value == 1
    for prec in (1, 2, 3):   # refinement and float precisions: not built for long systems
        assert L.bb_solve_batch_penta(hp, fake, other, 4, 4, prec, None) == -6
    assert L.bb_solve_batch_penta(hp, fake, fake, 4, 4, 4, None) == -1     # float rhs aliasing x
    assert L.bb_solve_batch_penta(hp, None, None, 0, 1, 4, None) == 0      # FP32 data: built
    assert L.bb_solve_batch_penta(hp, fake, fake, 4, 4, 0, None) == -6      # in place
    assert L.bb_solve_batch_penta_adjoint(hp, fake, fake, 4, 4, 0, None) == -6
    L.bb_factor_destroy(hp)
    ch = ctypes.c_void_p()
    sig, alp = ctypes.c_double(), ctypes.c_double()
    assert L.bb_factor_ch(4096, 2 * np.pi, 0.01, 1e-4, ctypes.byref(ch), ctypes.byref(sig),
                          ctypes.byref(alp)) == 0
    assert L.bb_ch_step(ch, fake, other, 4, 4, alp, 2, None) == -6          # one step per call
    assert L.bb_ch_step(ch, fake, fake, 4, 4, alp, 1, None) == -6           # in place
    ws = ctypes.c_void_p(0x3000)
    assert L.bb_ch_step_stats(ch, fake, other, 4, 4, alp, 1, 1, ws, ws, 1 << 20, None) == -6
    dx = 2 * np.pi / 4096
    assert L.bb_ch_forced_step(ch, fake, other, 4, 4, 1e-4, dx, ws, ws, ws, 2, None) == -6
    assert L.bb_ch_forced_step(ch, fake, fake, 4, 4, 1e-4, dx, ws, ws, ws, 1, None) == -6
    w5 = (ctypes.c_double * 5)(0.0, 0.0, 1.0, 0.0, 0.0)
    assert L.bb_cn_step(ch, w5, fake, other, 4, 4, 2, None) == -6           # one CN step per call
    assert L.bb_cn_step(ch, w5, fake, fake, 4, 4, 1, None) == -6            # in place
    L.bb_factor_destroy(ch)
    h = ctypes.c_void_p()
    assert L.bb_factor_shared_tri(None, None, None, 4, ctypes.byref(h)) == -1
    one = np.ones(4)
    assert L.bb_factor_shared_tri(_lib.dptr(one), _lib.dptr(one), _lib.dptr(one), 4, None) == -1


def test_solve_argument_checks_need_no_gpu(L):
    n = 16
    _, h = _factor(L, "tri", inputs.diffusion_tri_bands(n, 0.5), n)
    _, hp = _factor(L, "penta", inputs.hyperdiffusion_penta_bands(n, 0.25), n)
    fake = ctypes.c_void_p(0x1000)
    assert L.bb_solve_batch_tri(None, fake, fake, 4, 4, 0, None) == -1
    assert L.bb_solve_batch_tri(h, fake, fake, -1, 4, 0, None) == -1
    assert L.bb_solve_batch_tri(h, fake, fake, 8, 4, 0, None) == -1        # ld < m
    assert L.bb_solve_batch_tri(h, None, fake, 4, 4, 0, None) == -1
    assert L.bb_solve_batch_tri(h, fake, fake, 4, 4, 7, None) == -1        # bad precision
    assert L.bb_solve_batch_tri(h, fake, fake, 4, 4, 3, None) == -1        # float rhs aliasing double x
    assert L.bb_solve_batch_tri(h, fake, fake, 4, 4, 4, None) == -1        # the same, FP64 sweeps
    for prec in range(5):
        assert L.bb_plan(h, 1000, 0, prec, None, None, None, None) == 0
    assert L.bb_plan(h, 1000, 0, 5, None, None, None, None) == -1
    assert L.bb_solve_batch_penta(h, fake, fake, 4, 4, 0, None) == -1      # wrong kind
    assert L.bb_solve_batch_tri(hp, fake, fake, 4, 4, 0, None) == -1
    assert L.bb_solve_batch_tri_cyclic(h, fake, fake, 4, 4, 0, None) == -1  # not cyclic
    assert L.bb_ch_step(h, fake, fake, 4, 4, 1.0, 1, None) == -1           # not cyclic penta
    w3 = (ctypes.c_double * 3)(0.5, 0.0, 0.5)
    bad = (ctypes.c_double * 3)(0.5, float("nan"), 0.5)
    assert L.bb_ch_step_stats(h, fake, fake, 4, 4, 1.0, 4, 1, fake, fake, 1 << 20, None) == -1  # not cyclic penta
    _, hc = _factor(L, "penta_cyclic", inputs.ch_penta_bands(n, 0.3), n)
    assert L.bb_ch_step_stats(hc, fake, fake, 4, 4, 1.0, 4, 0, fake, fake, 1 << 20, None) == -1  # every < 1
    assert L.bb_ch_step_stats(hc, fake, fake, 4, 4, 1.0, 4, 1, None, fake, 1 << 20, None) == -1  # no lbar
    assert L.bb_ch_step_stats(hc, fake, fake, 4, 4, 1.0, 4, 1, fake, None, 1 << 20, None) == -1  # no workspace
    assert L.bb_ch_stats_workspace_bytes(hc, 4, 4) == 8 * 4             # one group of 4 runs, 4 samples
    assert L.bb_ch_step_stats(hc, fake, fake, 4, 4, 1.0, 4, 1, fake, fake, 8 * 4 - 1, None) == -1  # too small
    F = L.bb_ch_forced_step
    assert F(h, fake, fake, 4, 4, 0.1, 0.2, fake, fake, fake, 1, None) == -1    # not cyclic penta
    assert F(hc, fake, fake, 4, 4, 0.1, 0.2, None, fake, fake, 1, None) == -1   # no v
    assert F(hc, fake, fake, 4, 4, 0.1, 0.2, fake, fake, fake, 0, None) == -1   # steps < 1
    assert F(hc, fake, fake, 4, 4, -0.1, 0.2, fake, fake, fake, 1, None) == -1  # dt <= 0
    assert F(hc, fake, fake, 4, 4, 0.1, 0.0, fake, fake, fake, 1, None) == -1   # dx <= 0
    assert F(hc, fake, fake, 4, 4, float("inf"), 0.2, fake, fake, fake, 1, None) == -1
    assert F(hc, None, None, 0, 1, 0.1, 0.2, None, None, None, 1, None) == 0    # m = 0
    L.bb_factor_destroy(hc)
    assert L.bb_cn_step(h, None, fake, fake, 4, 4, 1, None) == -1           # no stencil
    assert L.bb_cn_step(h, bad, fake, fake, 4, 4, 1, None) == -1            # weight not finite
    assert L.bb_cn_step(h, w3, fake, fake, 4, 4, 0, None) == -1             # steps < 1
    assert L.bb_cn_step(h, w3, fake, fake, 8, 4, 1, None) == -1             # ld < m
    assert L.bb_cn_step(h, w3, None, None, 0, 1, 1, None) == 0              # m = 0: nothing to do
    assert L.bb_solve_batch_tri(h, None, None, 0, 1, 0, None) == 0         # m = 0: nothing to do
    assert L.bb_band_grad(h, fake, fake, 4, 4, None, None, 0, None) == -1
    assert L.bb_band_grad_noalloc(h, fake, fake, 4, 4, None, None) == -1   # no gradient
    assert L.bb_band_grad_noalloc(h, fake, fake, 8, 4, fake, None) == -1   # ld < m
    assert L.bb_band_grad_noalloc(None, fake, fake, 4, 4, fake, None) == -1
    assert L.bb_band_grad_noalloc(h, None, None, 0, 1, fake, None) == 0     # m = 0
    assert L.bb_solve_batch_tri_thread_per_system(hp, fake, fake, 4, 4, None) == -1
    A = L.bb_adjoint_band_grad
    big = 1 << 30
    lam = ctypes.c_void_p(0x100000)   # never dereferenced, far from fake's ranges
    assert A(None, fake, fake, lam, 4, 4, 1, fake, fake, big, None) == -1      # no factor
    assert A(h, fake, None, lam, 4, 4, 1, fake, fake, big, None) == -1        # no states
    assert A(h, fake, fake, lam, 4, 4, 1, None, fake, big, None) == -1        # no gradient
    assert A(h, fake, fake, lam, 4, 4, 0, fake, fake, big, None) == -1        # steps < 1
    assert A(h, fake, fake, lam, 8, 4, 1, fake, fake, big, None) == -1        # ld < m
    assert A(h, fake, fake, lam, 4, 4, 1, fake, fake, 0, None) == -1          # workspace too small
    assert A(h, fake, fake, lam, 4, 4, 1, fake, None, big, None) == -1        # no workspace
    assert A(h, None, None, None, 0, 1, 1, fake, None, 0, None) == 0          # m = 0
    inside = ctypes.c_void_p(0x1000 + 8 * 16 * 4)                             # traj's second state
    assert A(h, fake, fake, inside, 4, 4, 2, fake, fake, big, None) == -1     # lam inside traj
    L.bb_factor_destroy(h)
    L.bb_factor_destroy(hp)


def test_status_strings(L):
    for s in _lib.STATUS:
        assert L.bb_status_string(s)
    assert L.bb_status_string(12345) == b"unknown status"


def test_workspace_sizes(L):
    n = 64
    _, h = _factor(L, "tri", inputs.diffusion_tri_bands(n, 0.5), n)
    assert L.bb_band_grad_workspace_bytes(h, 0) == 0
    assert L.bb_band_grad_workspace_bytes(h, 1000) >= 3 * n * 8
    assert L.bb_mse_workspace_bytes(n, 1000) >= 8
    assert L.bb_band_grad_scratch_bytes() == 4 << 20
    L.bb_factor_destroy(h)


@pytest.mark.parametrize("kind,cyclic,n,m,fused", [
    ("tri", False, 1024, 65536, True), ("tri", True, 2048, 2500, True),
    ("penta", True, 1024, 20000, True), ("penta", False, 256, 5000, True),
    ("tri", False, 64, 33, False), ("penta", True, 1024, 2000, False),
    ("tri", False, 4096, 1000, False)])
def test_adjoint_band_grad_plan_and_workspace(L, kind, cyclic, n, m, fused):
    """Which path bb_adjoint_band_grad takes (host only) and its workspace:
    the groups' partial sums when fused, else one adjoint state plus the band
    gradient's partial sums."""
    bands = inputs.random_dominant_tri(n, 1) if kind == "tri" else inputs.random_dominant_penta(n, 1)
    name = kind + ("_cyclic" if cyclic else "")
    _, h = _factor(L, name, bands, n)
    nb = 3 if kind == "tri" else 5
    assert L.bb_adjoint_band_grad_fused(h, m) == int(fused)
    assert L.bb_adjoint_band_grad_fused(h, 0) == 0
    assert L.bb_adjoint_band_grad_workspace_bytes(h, 0, 1) == 0
    assert L.bb_adjoint_band_grad_workspace_bytes(h, m, m - 1) == 0       # ld < m
    ws = L.bb_adjoint_band_grad_workspace_bytes(h, m, m + 8)
    if fused:
        assert ws % (nb * n * 8) == 0 and nb * n * 8 * (m // 64) <= ws <= nb * n * 8 * m
    else:
        assert ws >= n * (m + 8) * 8 + L.bb_band_grad_workspace_bytes(h, m)
    L.bb_factor_destroy(h)


def _golden_ch_rows():
    path = os.path.join(ROOT, "tests", "golden", "ch_coefficients.txt")
    with open(path) as fh:
        return [tuple(float(x) for x in line.split()) for line in fh
                if line.strip() and not line.startswith("#")]


def test_cahn_hilliard_factor_coefficients(L):
    """bb_factor_ch: the library's own sigma = gamma dt / dx^4 and
    alpha = dt / dx^2 of the Section 5.1 scheme against the hand-evaluated
    golden values; host only."""
    for n, length, gamma, dt, s_ref, a_ref in _golden_ch_rows():
        h = ctypes.c_void_p()
        sigma, alpha = ctypes.c_double(), ctypes.c_double()
        assert L.bb_factor_ch(int(n), length, gamma, dt, ctypes.byref(h), ctypes.byref(sigma),
                              ctypes.byref(alpha)) == 0
        assert abs(sigma.value - s_ref) < 5e-6 * s_ref and abs(alpha.value - a_ref) < 5e-6 * a_ref
        nn, kind = ctypes.c_int64(), ctypes.c_int32()
        assert L.bb_factor_info(h, ctypes.byref(nn), ctypes.byref(kind), None) == 0
        assert (nn.value, kind.value) == (int(n), 3)
        L.bb_factor_destroy(h)
    h = ctypes.c_void_p()
    assert L.bb_factor_ch(4, 1.0, 0.01, 1e-3, ctypes.byref(h), None, None) == -1       # n < 5
    assert L.bb_factor_ch(64, -1.0, 0.01, 1e-3, ctypes.byref(h), None, None) == -1     # L <= 0
    assert L.bb_factor_ch(64, 1.0, 0.0, 1e-3, ctypes.byref(h), None, None) == -1       # gamma <= 0
    assert L.bb_factor_ch(64, 1.0, 0.01, float("nan"), ctypes.byref(h), None, None) == -1
    assert L.bb_factor_ch(64, 1.0, 0.01, 1e-3, None, None, None) == -1


def test_tuning_settings(L):
    """bb_set_tuning / bb_get_tuning: known names and valid values only, -1
    restores the automatic choice; host only."""
    for name, good, bad in [(b"max_chunk", 32, 48), (b"waves_per_system", 4, 3),
                            (b"waves_per_block", 2, 8), (b"lockstep", 0, 2),
                            (b"ch_uniform", 0, 5), (b"grid_linear", 1, -3),
                            (b"long_spread", 1, 2)]:
        assert L.bb_get_tuning(name) == -1
        assert L.bb_set_tuning(name, good) == 0 and L.bb_get_tuning(name) == good
        assert L.bb_set_tuning(name, bad) == -1 and L.bb_get_tuning(name) == good
        assert L.bb_set_tuning(name, -1) == 0 and L.bb_get_tuning(name) == -1
    assert L.bb_set_tuning(b"no_such_knob", 1) == -1
    assert b"unknown" in L.bb_last_error_message()
    assert L.bb_get_tuning(b"no_such_knob") == -2
    assert L.bb_set_tuning(None, 1) == -1
