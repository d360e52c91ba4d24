"""CPU model of the cross-lane schedules of the column kernel's chain sums
(a host-logic test: the moves are simulated on arrays of lanes, no GPU).

The reduce-scatter of the linear functionals keeps functional f's partial of
a lane at slot f ^ fl(seg), so that both partners of each halving move keep
their first half of slots and the moves are plain adds; the later moves add
the four entries left. The partner of each move is that of its DPP or LDS
control: xor 16, the row mirror (i <-> 15 - i), the half-row mirror
(i <-> 7 - i), quad xor 2 and quad xor 1. The test checks, for every segment
count the kernel instantiates, that the lane which stores functional f holds
the sum over the chain's lanes of their partials of f (exactly, with integer
data), and that the stored functionals cover each index once."""
import numpy as np
import pytest


def partner(kind, lane):
    if kind == 16:
        return lane ^ 16
    if kind == 8:
        return (lane & ~15) | (15 - (lane & 15))
    if kind == 4:
        return (lane & ~7) | (7 - (lane & 7))
    return lane ^ kind  # quad xor 2, 1


def g(kind, seg):
    b = [(seg >> i) & 1 for i in range(5)]
    return {16: b[4], 8: b[3], 4: b[3] ^ b[2], 2: b[2] ^ b[1], 1: b[2] ^ b[0]}[kind]


@pytest.mark.parametrize("S", [4, 8, 16, 32])
def test_select_free_reduce_scatter(S):
    NF = 8 if S == 32 else 4          # functionals per pass
    FB = NF.bit_length() - 1          # halving moves
    V = 4 * NF
    kinds = [S >> (j + 1) for j in range(S.bit_length() - 1)]
    rng = np.random.default_rng(S)
    part = rng.integers(-1000, 1000, size=(S, NF, 4))  # partial[lane][f][k]
    fl = [0] * S
    for seg in range(S):
        for j in range(FB):
            fl[seg] = (fl[seg] << 1) | g(kinds[j], seg)
    # slot p of a lane holds functional p >> 2 xor fl, component p & 3
    v = np.zeros((S, V), dtype=np.int64)
    for seg in range(S):
        for fp in range(NF):
            v[seg, 4 * fp:4 * fp + 4] = part[seg, fp ^ fl[seg]]
    for j, kind in enumerate(kinds):
        new = v.copy()
        for seg in range(S):
            p = partner(kind, seg)
            assert 0 <= p < S
            if j < FB:
                hh = V >> (j + 1)
                new[seg, :hh] = v[seg, :hh] + v[p, hh:2 * hh]
            else:
                new[seg, :4] = v[seg, :4] + v[p, :4]
        v = new
    total = part.sum(axis=0)
    stored = {}
    for seg in range(S):
        if seg & ((S >> FB) - 1) == 0:
            assert fl[seg] not in stored
            stored[fl[seg]] = v[seg, :4]
            assert np.array_equal(v[seg, :4], total[fl[seg]]), (seg, fl[seg])
    assert sorted(stored) == list(range(NF))


@pytest.mark.parametrize("S", [16, 32])
def test_branch_free_scan_steps_take_exactly_the_dpp_sources(S):
    """With 16 or 32 segments, a chain lane takes a scan step (row shift by o)
    exactly when the DPP move has a source lane within the row: the lanes
    without one receive the identity map instead of a branch."""
    for lane in range(64):
        seg = lane & (S - 1)
        for o in (1, 2, 4, 8):
            if o >= S:
                continue
            take_fwd = seg >= o and (lane & 15) >= o
            assert take_fwd == ((lane & 15) - o >= 0)
            take_bwd = seg + o < S and (lane & 15) + o < 16
            assert take_bwd == ((lane & 15) + o < 16)
