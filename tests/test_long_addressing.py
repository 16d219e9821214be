"""CPU replay of the addressing of the small-batch long-system scan
(long_scan_spread in csrc/long_core.h): for the shapes the GPU tests and
benchmarks run, every access to the solution array (the launch sequence's
scratch) stays inside the n x ld array at the lane's own column, every chunk
index inside the full chunks, every chunk-matrix index inside the table's
P K^2 entries, and no block stores a chunk that a later block loads before
it was meant to.  The formulas restate the kernel's: lane l of a forward
block j0 holds chunk j0 + l, of a backward block jt chunk jt - l, loads for
the next two blocks clamped to the full chunks."""
import itertools

import pytest

W = 64


def replay(n, m, ld, C, K, cyclic):
    P = (n + C - 1) // C
    full = P - 1
    assert full >= 1 and 3 * K <= C
    MK = P * K * K
    stored_fwd = set()

    def touch(row, k):
        assert 0 <= row < n and 0 <= k < m and row * ld + k < n * ld

    def mat(j):
        assert 0 <= j < full and j * K * K + K * K <= MK

    for k in sorted({0, m - 1}):
        fwd_at = lambda j: j if j < full else full - 1
        for lane in range(W):                 # the first two blocks
            for j in (fwd_at(lane), fwd_at(W + lane)):
                touch(j * C, k), K == 2 and touch(j * C + 1, k), mat(j)
        j0 = 0
        while j0 < full:
            cnt = min(full - j0, W)
            for lane in range(W):
                j = fwd_at(j0 + 2 * W + lane)
                touch(j * C, k), mat(j)
                if j0 + 2 * W + lane < full:  # a real chunk: not stored yet
                    assert (k, j) not in stored_fwd
                if lane < cnt:
                    touch((j0 + lane) * C, k), K == 2 and touch((j0 + lane) * C + 1, k)
                    stored_fwd.add((k, j0 + lane))
            j0 += W
        assert all((k, j) in stored_fwd for j in range(full))
        assert 1 <= n - full * C <= C        # the tail: rows full*C .. n-1
        bwd_at = lambda j: j if j >= 0 else 0
        for lane in range(W):
            for j in (bwd_at(full - 1 - lane), bwd_at(full - 1 - W - lane)):
                [touch(j * C + r, k) for r in range(2 * K)]
                mat(j)
        jt = full - 1
        while jt >= 0:
            cnt = min(jt + 1, W)
            for lane in range(W):
                j = bwd_at(jt - 2 * W - lane)
                [touch(j * C + r, k) for r in range(2 * K)]
                mat(j)
                if lane < cnt:
                    assert 0 <= jt - lane < full
                    [touch((jt - lane) * C + r, k) for r in range(K, 2 * K)]
            jt -= W
        if cyclic:
            for lane in range(W):
                for j in range(lane, full, W):
                    [touch(j * C + r, k) for r in range(2 * K, 3 * K)]


SHAPES = [(2049, 70), (4096, 64), (8192, 1), (5000, 200), (16384, 3), (1025, 65), (4096, 33),
          (8192, 64), (3001, 129), (16384, 2), (4097, 100), (2050, 100), (3000, 150),
          (16384, 512), (262144, 1), (2048, 4095)]


@pytest.mark.parametrize("n,m", SHAPES)
def test_spread_scan_addressing_in_bounds(n, m):
    for C, K, cyclic in itertools.product((16, 32, 64), (1, 2), (False, True)):
        if (K == 1 and n <= 2048) or (K == 2 and n <= 1024):
            continue
        replay(n, m, m + 21, C, K, cyclic)
