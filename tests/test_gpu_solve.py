"""GPU parity: every solve path of libbandbatch against the FP64 oracle, element
by element on the same seeded inputs, at sizes that span several chunks, a
ragged last chunk, a ragged batch tail and the degenerate sizes.

Bars: FP64 1e-12, FP32 sweeps + one FP64-residual refinement 1e-10 (per-system
relative 2-norm error, max over systems); unrefined FP32 only as a sanity check."""
import numpy as np
import pytest
import torch

import oracle
from paper_2107_05395_amd import inputs
from tests.gpu_util import dev, host, rel_err, say

pytestmark = pytest.mark.gpu

# sigma of the Section 5.1 Cahn-Hilliard matrix at n = 256, L = 2 pi,
# gamma = 0.01, dt = 1e-3 (a parameter of a test matrix with kappa ~ 441)
CH_SIGMA_256 = 27.5575

F64_TOL = 1e-12
F32R_TOL = 1e-10
F32_TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    from paper_2107_05395_amd import solver  # noqa: F401  (fails loudly if not built)
    oracle.build()
    torch.cuda.synchronize()


def make(kind, n, seed, cyclic=False, dominant=True):
    from paper_2107_05395_amd import Factor
    if kind == "tri":
        bands = inputs.random_dominant_tri(n, seed) if dominant else inputs.diffusion_tri_bands(n, 0.5)
        return Factor.tri(*bands, cyclic=cyclic), bands
    bands = inputs.random_dominant_penta(n, seed) if dominant else inputs.hyperdiffusion_penta_bands(n, 0.25)
    return Factor.penta(*bands, cyclic=cyclic), bands


def oracle_solve(kind, bands, rhs, cyclic):
    if kind == "tri":
        return oracle.tri_solve(*bands, rhs, cyclic=cyclic)
    return oracle.penta_solve(*bands, rhs, cyclic=cyclic)


def oracle_adjoint(kind, bands, g, cyclic):
    if kind == "tri":
        return oracle.tri_adjoint(*bands, g, cyclic=cyclic)
    return oracle.penta_adjoint(*bands, g, cyclic=cyclic)


SHAPES_TRI = [(1, 5), (2, 3), (3, 64), (5, 65), (8, 1), (63, 130), (64, 64), (100, 77),
              (256, 1024), (257, 300), (512, 200), (1000, 129), (1024, 64), (1025, 40), (2048, 33)]
SHAPES_PENTA = [(1, 3), (2, 4), (3, 9), (4, 64), (5, 70), (9, 33), (64, 100), (130, 65),
                (256, 128), (1000, 50), (1024, 96)]


@pytest.mark.parametrize("n,m", SHAPES_TRI)
def test_tri_f64(n, m):
    say("tri f64", n, m)
    f, bands = make("tri", n, seed=n)
    rhs = inputs.uniform_batch(n, m, seed=1000 + n)
    x = host(f.solve(dev(rhs)))
    assert rel_err(x, oracle.tri_solve(*bands, rhs)) < F64_TOL


@pytest.mark.parametrize("n,m", SHAPES_PENTA)
def test_penta_f64(n, m):
    say("penta f64", n, m)
    f, bands = make("penta", n, seed=n)
    rhs = inputs.uniform_batch(n, m, seed=2000 + n)
    x = host(f.solve(dev(rhs)))
    assert rel_err(x, oracle.penta_solve(*bands, rhs)) < F64_TOL


@pytest.mark.parametrize("kind,n,m", [("tri", 3, 10), ("tri", 4, 64), ("tri", 97, 130),
                                      ("tri", 256, 256), ("tri", 1000, 70), ("tri", 2048, 17),
                                      ("penta", 5, 10), ("penta", 6, 64), ("penta", 77, 100),
                                      ("penta", 256, 256), ("penta", 1000, 40),
                                      ("penta", 1024, 12)])
def test_cyclic_f64(kind, n, m):
    say("cyclic f64", kind, n, m)
    f, bands = make(kind, n, seed=3 * n, cyclic=True)
    rhs = inputs.uniform_batch(n, m, seed=3000 + n)
    x = host(f.solve(dev(rhs)))
    assert rel_err(x, oracle_solve(kind, bands, rhs, True)) < F64_TOL


@pytest.mark.parametrize("kind", ["tri", "penta"])
@pytest.mark.parametrize("cyclic", [False, True])
@pytest.mark.parametrize("n", [64, 300, 1024])
def test_refine_f32r(kind, cyclic, n):
    say("f32r", kind, cyclic, n)
    f, bands = make(kind, n, seed=7 * n, cyclic=cyclic, dominant=False)
    rhs = inputs.uniform_batch(n, 200, seed=4000 + n)
    x = host(f.solve(dev(rhs), precision="f32r"))
    err = rel_err(x, oracle_solve(kind, bands, rhs, cyclic))
    say("  rel err", err)
    assert err < F32R_TOL


@pytest.mark.parametrize("kind", ["tri", "penta"])
@pytest.mark.parametrize("cyclic", [False, True])
@pytest.mark.parametrize("n", [64, 300, 512, 1024])
def test_refine_f32_rhs(kind, cyclic, n):
    """FP32 right-hand-side data, double solution: against the oracle solving
    with the same (float) values promoted to double."""
    say("f32rhs", kind, cyclic, n)
    f, bands = make(kind, n, seed=9 * n, cyclic=cyclic, dominant=False)
    rhs32 = inputs.uniform_batch(n, 333, seed=4500 + n).astype(np.float32)
    t = dev(rhs32, torch.float32)
    x = f.solve(t, precision="f32rhs")
    assert x.dtype == torch.float64
    err = rel_err(host(x), oracle_solve(kind, bands, rhs32.astype(np.float64), cyclic))
    say("  rel err", err)
    assert err < F32R_TOL
    lam = host(f.adjoint(t, precision="f32rhs"))
    assert rel_err(lam, oracle_adjoint(kind, bands, rhs32.astype(np.float64), cyclic)) < F32R_TOL


@pytest.mark.parametrize("kind", ["tri", "penta"])
@pytest.mark.parametrize("cyclic", [False, True])
@pytest.mark.parametrize("n,m", [(5, 70), (64, 333), (300, 1000), (1024, 70000), (2048, 3000)])
def test_f32_rhs_f64_sweeps(kind, cyclic, n, m):
    """FP32 right-hand-side data solved with the FP64 sweeps: the FP64 solve
    of the promoted values, to the FP64 bar (1e-12 against the oracle on the
    same promoted values), and bitwise the FP64 solve of the promoted array
    (same decomposition and arithmetic); the adjoint likewise."""
    if kind == "penta" and n > 1024:
        pytest.skip("long pentadiagonal systems take the FP64 three-launch path only")
    say("f32rhs_f64", kind, cyclic, n, m)
    f, bands = make(kind, n, seed=13 * n, cyclic=cyclic, dominant=False)
    rhs32 = inputs.uniform_batch(n, m, seed=4700 + n).astype(np.float32)
    t = dev(rhs32, torch.float32)
    x = f.solve(t, precision="f32rhs_f64")
    assert x.dtype == torch.float64
    assert rel_err(host(x), oracle_solve(kind, bands, rhs32.astype(np.float64), cyclic)) < 1e-12
    assert torch.equal(x, f.solve(t.double(), precision="f64"))
    lam = f.adjoint(t, precision="f32rhs_f64")
    assert torch.equal(lam, f.adjoint(t.double(), precision="f64"))


@pytest.mark.parametrize("kind", ["tri", "penta"])
@pytest.mark.parametrize("cyclic", [False, True])
def test_plain_f32(kind, cyclic):
    n = 512
    f, bands = make(kind, n, seed=11, cyclic=cyclic, dominant=False)
    rhs = inputs.uniform_batch(n, 100, seed=12)
    x = host(f.solve(dev(rhs, torch.float32), precision="f32"))
    assert rel_err(x, oracle_solve(kind, bands, rhs, cyclic)) < F32_TOL


@pytest.mark.parametrize("kind", ["tri", "penta"])
@pytest.mark.parametrize("cyclic", [False, True])
@pytest.mark.parametrize("n", [5, 64, 257, 1024])
def test_adjoint(kind, cyclic, n):
    say("adjoint", kind, cyclic, n)
    f, bands = make(kind, n, seed=13 * n, cyclic=cyclic)
    g = inputs.uniform_batch(n, 90, seed=5000 + n)
    ref = oracle_adjoint(kind, bands, g, cyclic)
    assert rel_err(host(f.adjoint(dev(g))), ref) < F64_TOL
    assert rel_err(host(f.adjoint(dev(g), precision="f32r")), ref) < F32R_TOL


def test_in_place_and_strided():
    n, m, ld = 300, 100, 160
    f, bands = make("penta", n, seed=1)
    big = inputs.uniform_batch(n, ld, seed=6)
    t = dev(big)
    view = t[:, :m]
    f.solve(view, out=view)                      # in place on a strided view
    out = host(t)
    assert rel_err(out[:, :m], oracle.penta_solve(*bands, big[:, :m])) < F64_TOL
    assert np.array_equal(out[:, m:], big[:, m:])  # columns past m untouched


def test_out_of_place_leaves_input():
    n, m = 256, 500
    f, _ = make("tri", n, seed=2)
    rhs = inputs.uniform_batch(n, m, seed=7)
    t = dev(rhs)
    f.solve(t)
    assert np.array_equal(host(t), rhs)


def test_empty_batch_is_noop():
    f, _ = make("tri", 64, seed=3)
    t = torch.zeros(64, 0, dtype=torch.float64, device="cuda")
    f.solve(t)
    torch.cuda.synchronize()


def test_thread_per_system_baseline():
    n, m = 512, 3000
    f, bands = make("tri", n, seed=4)
    rhs = inputs.uniform_batch(n, m, seed=8)
    assert rel_err(host(f.solve_thread_per_system(dev(rhs))), oracle.tri_solve(*bands, rhs)) < F64_TOL
    t = dev(rhs)
    f.solve_thread_per_system(t, out=t)          # the paper's in-place form
    assert rel_err(host(t), oracle.tri_solve(*bands, rhs)) < F64_TOL


def test_bitwise_deterministic():
    n, m = 1024, 4096
    f, _ = make("penta", n, seed=5, cyclic=True)
    t = dev(inputs.uniform_batch(n, m, seed=9))
    a = host(f.solve(t))
    b = host(f.solve(t))
    assert np.array_equal(a, b)


def test_factor_on_the_oracle_matrices_of_every_config():
    """The LHS of each configured workload, small batch, against the oracle."""
    for kind, n, bands, cyc in [
        ("tri", 256, inputs.diffusion_tri_bands(256, 0.5), False),
        ("tri", 512, inputs.diffusion_tri_bands(512, 1.0), False),
        ("penta", 1024, inputs.hyperdiffusion_penta_bands(1024, 0.25), False),
        ("penta", 256, inputs.ch_penta_bands(256, CH_SIGMA_256), True),
        ("tri", 1024, inputs.variable_diffusion_bands(inputs.rng(1).uniform(0.5, 1.5, 1024), 0.5), False),
    ]:
        from paper_2107_05395_amd import Factor
        f = Factor.tri(*bands, cyclic=cyc) if kind == "tri" else Factor.penta(*bands, cyclic=cyc)
        rhs = inputs.uniform_batch(n, 256, seed=n)
        ref = oracle_solve(kind, bands, rhs, cyc)
        say("config matrix", kind, n, cyc)
        assert rel_err(host(f.solve(dev(rhs))), ref) < F64_TOL
        assert rel_err(host(f.solve(dev(rhs), precision="f32r")), ref) < F32R_TOL


@pytest.mark.parametrize("kind,n,cyclic", [("tri", 512, False), ("tri", 1024, True),
                                           ("tri", 2048, False), ("penta", 512, True),
                                           ("penta", 1024, False), ("penta", 1024, True),
                                           ("tri", 1000, True), ("tri", 1500, False),
                                           ("penta", 600, True), ("penta", 1000, False),
                                           ("tri", 1536, True)])
@pytest.mark.parametrize("rows", [64, 128, 32])
def test_split_groups_match_single_wave_groups(kind, n, cyclic, rows, tuning):
    """A system group spread over 2, 4 or 8 waves (boundary states exchanged
    through LDS) computes exactly what a one-wave group computes: same
    operations in the same order, so the results are bitwise equal.  Solve,
    adjoint, plain FP32 and FP32 + refinement; 64 rows per lane (the default
    for large batches), 128 rows and 32 rows (refinement groups of up to 8
    waves; a width a kernel cannot run falls back to the automatic one)."""
    tuning.set("max_chunk", str(rows))
    f, bands = make(kind, n, seed=17 * n, cyclic=cyclic)
    m = 1000                                   # not a multiple of any group width
    rhs = inputs.uniform_batch(n, m, seed=6000 + n)
    ref = oracle_solve(kind, bands, rhs, cyclic)
    t = dev(rhs)
    got = {}
    for q in (1, 2, 4, 8):
        tuning.set("waves_per_system", str(q))
        say("split", kind, n, cyclic, "waves per system", q)
        got[q] = host(f.solve(t))
        assert rel_err(got[q], ref) < F64_TOL
        lam = host(f.adjoint(t))
        assert rel_err(lam, oracle_adjoint(kind, bands, rhs, cyclic)) < F64_TOL
        x32 = host(f.solve(dev(rhs, torch.float32), precision="f32"))
        assert rel_err(x32, ref) < F32_TOL
        got[("r", q)] = host(f.solve(t, precision="f32r"))
        assert rel_err(got[("r", q)], ref) < F32R_TOL
    tuning.set("waves_per_system", "2")
    assert np.array_equal(host(f.solve(t, precision="f32r")), got[("r", 2)])   # repeatable
    for q in (2, 4):
        say("  max |f32r diff| q=1 vs q=%d" % q, np.max(np.abs(got[("r", 1)] - got[("r", q)])))
    assert all(np.array_equal(got[1], got[q]) for q in (2, 4, 8))
    assert np.array_equal(got[("r", 1)], got[("r", 2)])
    assert np.array_equal(got[("r", 1)], got[("r", 4)])


@pytest.mark.parametrize("n,m,rows", [(256, 1024, 32), (64, 4096, 16), (1024, 64, 32),
                                      (2048, 256, 64)])
def test_small_batches_take_short_chunks(n, m, rows, tuning):
    """With fewer than 2^16 lanes of 64-row chunks the solve takes the
    latency rule's chunk (the power of two >= 2 sqrt(n), at most 32, at most
    32 chunks per system): bitwise what forcing that chunk gives, and within
    the FP64 tolerance of the oracle."""
    f, bands = make("tri", n, seed=n + m)
    assert f.plan(m)["chunk"] == rows
    rhs = inputs.uniform_batch(n, m, seed=n + m + 1)
    t = dev(rhs)
    auto = host(f.solve(t))
    assert rel_err(auto, oracle_solve("tri", bands, rhs, False)) < F64_TOL
    tuning.set("max_chunk", str(rows))
    assert np.array_equal(auto, host(f.solve(t)))


def test_workgroup_shape_and_lockstep_do_not_change_results(tuning):
    """Waves per workgroup and the lockstep barrier only change which waves run
    together, not the arithmetic: bitwise equal results (ragged n, so the
    groups are one wave each)."""
    n, m = 300, 777
    f, bands = make("penta", n, seed=31, cyclic=True)
    rhs = inputs.uniform_batch(n, m, seed=32)
    t = dev(rhs)
    outs = []
    for w in ("1", "2", "4"):
        for lock in ("0", "1"):
            tuning.set("waves_per_block", w)
            tuning.set("lockstep", lock)
            outs.append(host(f.solve(t)))
    assert rel_err(outs[0], oracle_solve("penta", bands, rhs, True)) < F64_TOL
    assert all(np.array_equal(o, outs[0]) for o in outs[1:])


# ---------------------------------------------------------------- hard matrices
def _dense(kind, bands, n, cyclic):
    A = np.zeros((n, n))
    K = 1 if kind == "tri" else 2
    for q, band in enumerate(bands):
        off = q - K
        for i in range(n):
            j = i + off
            if cyclic:
                A[i, j % n] += band[i]
            elif 0 <= j < n:
                A[i, j] = band[i]
    return A


def _hard(name, n, seed):
    """Matrices near the edge of what an LU without pivoting handles:
    weakly diagonally dominant random bands (margin 1e-3, non-symmetric),
    and implicit Euler diffusion with r = 1000 (kappa about 4000)."""
    if name == "weak_tri":
        return "tri", inputs.random_dominant_tri(n, seed, margin=1e-3)
    if name == "weak_penta":
        return "penta", inputs.random_dominant_penta(n, seed, margin=1e-3)
    if name == "diffusion_r1000":
        return "tri", inputs.diffusion_tri_bands(n, 1000.0)
    assert name == "hyperdiffusion_r1000"
    return "penta", inputs.hyperdiffusion_penta_bands(n, 1000.0)


@pytest.mark.parametrize("name,n", [("weak_tri", 2048), ("weak_penta", 1024),
                                    ("diffusion_r1000", 2048), ("hyperdiffusion_r1000", 1024)])
@pytest.mark.parametrize("cyclic", [False, True])
def test_hard_matrices(name, n, cyclic, tuning):
    """64-row chunks (the decomposition whose chunk-transfer weights decay
    slowest on these matrices), FP64 and FP32 + refinement.  Tolerances from
    the arithmetic: FP64 max(1e-12, 2 kappa u); one refinement step leaves
    about (kappa u32)^2 + kappa u of the first solve's error, taken with a
    factor 4."""
    tuning.set("max_chunk", "64")
    kind, bands = _hard(name, n, seed=n + 17)
    from paper_2107_05395_amd import Factor
    f = Factor.tri(*bands, cyclic=cyclic) if kind == "tri" else Factor.penta(*bands, cyclic=cyclic)
    assert f.plan(300)["chunk"] == 64
    kappa = float(np.linalg.cond(_dense(kind, bands, n, cyclic)))
    rhs = inputs.uniform_batch(n, 300, seed=n + 18)
    ref = oracle_solve(kind, bands, rhs, cyclic)
    u, u32 = 2.0 ** -53, 2.0 ** -24
    tol64 = max(F64_TOL, 2.0 * kappa * u)
    tol32r = max(F32R_TOL, 4.0 * ((kappa * u32) ** 2 + kappa * u))
    e64 = rel_err(host(f.solve(dev(rhs))), ref)
    e32 = rel_err(host(f.solve(dev(rhs), precision="f32r")), ref)
    say("hard", name, n, cyclic, "kappa %.3g" % kappa, "f64", e64, tol64, "f32r", e32, tol32r)
    assert e64 < tol64
    assert e32 < tol32r
    lam = host(f.adjoint(dev(rhs)))
    assert rel_err(lam, oracle_adjoint(kind, bands, rhs, cyclic)) < tol64
