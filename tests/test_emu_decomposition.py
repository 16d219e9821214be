"""CPU check of the chunked decomposition the GPU sweep uses.

tests/emu/chunk_emu.cpp builds the library's own host factor and coefficient
tables and replays one wave's dataflow for one system in double on the CPU
(boundary-state weights, scans over chunks, forward and backward passes,
periodic correction).  Its result must equal the oracle's for every matrix
kind, direction, chunk size and a ragged last chunk -- so a mistake in the
table construction or the scan algebra shows up here, without a GPU."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2107_05395_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "emu", "chunk_emu.cpp")
FACTOR = os.path.join(ROOT, "paper_2107_05395_amd", "csrc", "factor.cpp")
LIB = os.path.join(HERE, "emu", "libchunk_emu.so")


@pytest.fixture(scope="module")
def emu():
    newest = max(os.path.getmtime(p) for p in (SRC, FACTOR,
                 os.path.join(ROOT, "paper_2107_05395_amd", "csrc", "internal.h"),
                 os.path.join(ROOT, "paper_2107_05395_amd", "csrc", "factor.h")))
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        tmp = LIB + ".tmp%d" % os.getpid()
        # host-only build: no device code in either file
        subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", "-fPIC", "-shared", SRC, FACTOR,
                        "-o", tmp], check=True)
        os.replace(tmp, LIB)
    lib = ctypes.CDLL(LIB)
    P = ctypes.POINTER(ctypes.c_double)
    lib.emu_solve.argtypes = [ctypes.c_int] + [P] * 5 + [ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P]
    lib.emu_solve_long.argtypes = lib.emu_solve.argtypes
    lib.emu_solve_long_spread.argtypes = lib.emu_solve.argtypes
    return lib


def run(emu, kind_id, bands, n, adjoint, C, f, entry="emu_solve"):
    bands = [np.ascontiguousarray(b, dtype=np.float64) for b in bands] + [np.zeros(n)] * (5 - len(bands))
    f = np.ascontiguousarray(f, dtype=np.float64)
    x = np.empty(n)
    P = ctypes.POINTER(ctypes.c_double)
    st = getattr(emu, entry)(kind_id, *(b.ctypes.data_as(P) for b in bands), n, adjoint, C,
                             f.ctypes.data_as(P), x.ctypes.data_as(P))
    assert st == 0, st
    return x


CASES = [(n, C) for n in (4, 5, 7, 16, 33, 64, 100, 256, 257, 1000) for C in (4, 8, 16, 64)
         if (n + C - 1) // C <= 64]


@pytest.mark.parametrize("kind", ["tri", "tri_cyclic", "penta", "penta_cyclic"])
@pytest.mark.parametrize("adjoint", [0, 1])
@pytest.mark.parametrize("n,C", CASES)
def test_chunked_decomposition_matches_oracle(emu, oracle, kind, adjoint, n, C):
    cyclic = kind.endswith("cyclic")
    penta = kind.startswith("penta")
    if cyclic and n < (5 if penta else 3):
        pytest.skip("below the periodic minimum size")
    kind_id = {"tri": 0, "tri_cyclic": 1, "penta": 2, "penta_cyclic": 3}[kind]
    bands = inputs.random_dominant_penta(n, seed=n + C) if penta else inputs.random_dominant_tri(n, seed=n + C)
    f = inputs.uniform_batch(n, 1, seed=7 * n + C)[:, 0]
    x = run(emu, kind_id, bands, n, adjoint, C, f)
    if penta:
        ref = (oracle.penta_adjoint if adjoint else oracle.penta_solve)(*bands, f[:, None], cyclic=cyclic)[:, 0]
    else:
        ref = (oracle.tri_adjoint if adjoint else oracle.tri_solve)(*bands, f[:, None], cyclic=cyclic)[:, 0]
    assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref)


LONG_CASES = [(n, C) for n in (17, 33, 48, 100, 257, 1000, 1025, 4097) for C in (16, 32, 64)
              if (n + C - 1) // C >= 2]


@pytest.mark.parametrize("kind", ["tri", "tri_cyclic", "penta", "penta_cyclic"])
@pytest.mark.parametrize("adjoint", [0, 1])
@pytest.mark.parametrize("n,C", LONG_CASES)
def test_long_system_launches_match_oracle(emu, oracle, kind, adjoint, n, C):
    """The reduce / scan / solve sequence of long systems, with the solution
    array as scratch, replayed from the library's tables: any number of
    chunks, a tail of 1 .. C rows."""
    cyclic = kind.endswith("cyclic")
    penta = kind.startswith("penta")
    kind_id = {"tri": 0, "tri_cyclic": 1, "penta": 2, "penta_cyclic": 3}[kind]
    bands = inputs.random_dominant_penta(n, seed=n + C) if penta else inputs.random_dominant_tri(n, seed=n + C)
    f = inputs.uniform_batch(n, 1, seed=11 * n + C)[:, 0]
    x = run(emu, kind_id, bands, n, adjoint, C, f, entry="emu_solve_long")
    if penta:
        ref = (oracle.penta_adjoint if adjoint else oracle.penta_solve)(*bands, f[:, None], cyclic=cyclic)[:, 0]
    else:
        ref = (oracle.tri_adjoint if adjoint else oracle.tri_solve)(*bands, f[:, None], cyclic=cyclic)[:, 0]
    assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind", ["tri", "tri_cyclic", "penta", "penta_cyclic"])
@pytest.mark.parametrize("adjoint", [0, 1])
@pytest.mark.parametrize("n,C", [(33, 16), (100, 16), (1000, 16), (1040, 16), (1041, 16),
                                 (2049, 16), (4097, 16), (8192, 32), (16000, 32), (16384, 32),
                                 (9000, 64)])
def test_long_system_spread_scan_matches_oracle(emu, oracle, kind, adjoint, n, C):
    """The small-batch scan (blocks of 64 chunks whose affine maps are scanned
    across the wave) replayed on the host against the oracle: one to eight
    blocks, a last block of 1 .. 64 chunks, tails of 1 .. C rows."""
    cyclic = kind.endswith("cyclic")
    penta = kind.startswith("penta")
    kind_id = {"tri": 0, "tri_cyclic": 1, "penta": 2, "penta_cyclic": 3}[kind]
    bands = inputs.random_dominant_penta(n, seed=n + C) if penta else inputs.random_dominant_tri(n, seed=n + C)
    f = inputs.uniform_batch(n, 1, seed=13 * n + C)[:, 0]
    x = run(emu, kind_id, bands, n, adjoint, C, f, entry="emu_solve_long_spread")
    if penta:
        ref = (oracle.penta_adjoint if adjoint else oracle.penta_solve)(*bands, f[:, None], cyclic=cyclic)[:, 0]
    else:
        ref = (oracle.tri_adjoint if adjoint else oracle.tri_solve)(*bands, f[:, None], cyclic=cyclic)[:, 0]
    assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref)
