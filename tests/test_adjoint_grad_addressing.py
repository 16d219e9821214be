"""CPU replay of the band-gradient reduction of the fused adjoint kernel
(adjoint_grad_kernel.h) for every geometry it is built for: each lane's
products of one row block go through the halving rounds (v_permlane32_swap /
v_permlane16_swap pairings and the shuffle-and-select rounds, replayed on
sets of (slot, value) labels), the staging writes and the per-entry sums.
Every (chunk, row, band) entry of the block must receive the contribution of
each of the group's S systems exactly once, every staging write must land in
the wave's area and no two writes may share an address.  The formulas
restate the kernel's: lane = chunk-in-wave * S + slot, value index
v = row * (2K+1) + band, halving round r pairs slot bit SL-r and keeps half
V >> r of the values, staging index h * (E+1) + chunk * V + offset + i."""
import itertools

import pytest

WAVE = 64


def geometry(K, SL):
    S = 1 << SL
    W = WAVE // S
    cap = 8 if K == 1 else 4
    fit = (16 if K == 1 else 8) * S // WAVE
    RB = min(cap, fit)
    NH = 2 if (SL == 6 or K == 2) else 1
    NB = 2 * K + 1
    V = RB * NB
    return S, W, RB, NH, NB, V


def halve(vals, X, lane_of):
    """One halving round across lane bit X on per-lane lists of value sets."""
    out = {}
    for lane, v in vals.items():
        N = len(v)
        H = N // 2
        partner = lane ^ X
        top = (lane & X) != 0
        keep = v[H:] if top else v[:H]
        send = vals[partner][H:] if top else vals[partner][:H]   # partner sends the half we keep
        out[lane] = [a | b for a, b in zip(keep, send)]
    return out


@pytest.mark.parametrize("K,SL", [(1, 4), (1, 5), (1, 6), (2, 5), (2, 6)])
def test_reduction_covers_every_entry_once(K, SL):
    S, W, RB, NH, NB, V = geometry(K, SL)
    HS, E = S >> NH, W * V
    EP = E + 1
    assert E <= WAVE and (V >> NH) << NH == V
    # lane l holds, for value index v, the set {(slot, chunk, v)}: one product
    vals = {}
    for lane in range(WAVE):
        wl, sl = lane >> SL, lane & (S - 1)
        vals[lane] = [frozenset({(sl, wl, v)}) for v in range(V)]
    for r in range(1, NH + 1):
        vals = halve(vals, S >> r, None)
    stage = {}
    for lane in range(WAVE):
        wl, sl = lane >> SL, lane & (S - 1)
        h = sl & (HS - 1)
        off = sum(((sl >> (SL - r)) & 1) * (V >> r) for r in range(1, NH + 1))
        for i, val in enumerate(vals[lane]):
            addr = h * EP + wl * V + off + i
            assert 0 <= addr < HS * EP
            assert addr not in stage, (lane, i)
            stage[addr] = val
    for e in range(E):
        wl_e, v_e = e // V, e % V
        got = []
        for s in range(HS):
            got.extend(stage[s * EP + e])
        # every slot of the chunk, once, for this entry's value index
        assert sorted(got) == [(sl, wl_e, v_e) for sl in range(S)], (e, got[:4])


@pytest.mark.parametrize("K,SL", [(1, 4), (1, 5), (1, 6), (2, 5), (2, 6)])
def test_block_entries_map_to_rows_and_bands(K, SL):
    """The entry a summing lane owns names a distinct (chunk, row, band) of
    the block, and the blocks of a chunk tile its rows."""
    S, W, RB, NH, NB, V = geometry(K, SL)
    E = W * V
    seen = set()
    for e in range(E):
        wl_e, v_e = e // V, e % V
        r_e, q_e = v_e // NB, v_e % NB
        assert 0 <= wl_e < W and 0 <= r_e < RB and 0 <= q_e < NB
        seen.add((wl_e, r_e, q_e))
    assert len(seen) == E
    for C in (32, 64):
        rows = sorted(b * RB + r for b, r in itertools.product(range(C // RB), range(RB)))
        assert rows == list(range(C))
