"""The Jacobi block-pair schedule (host logic, no GPU): lyap_jacobi_schedule through the C ABI.

The spectral decompositions (Fragments 2.1-2.4, Alg 3.2) sweep block pairs in the modulus
ordering.  Checked here: every round is a perfect matching of the nb blocks; each block pair
is a real pair exactly once per sweep; the pseudo-pair of even rounds is the two idle blocks;
the map from blocks to pairs is consistent; every block is in a real pair in round 0 or 1
(those rounds give full subproblem sweeps); and, over several sweeps, the pairs that share a
block come in exactly the row-cyclic order (pair (i, j) of row-cyclic sweep s sits in round
i + j + s nb), which is what makes the parallel schedule apply the rotations of row-cyclic
Jacobi."""
import itertools

import numpy as np
import pytest

import paper_2510_02126_amd as lyap
from paper_2510_02126_amd import _lib


@pytest.mark.parametrize("nb", [2, 4, 6, 8, 16, 30, 128, 256])
def test_rounds_are_matchings_and_sweeps_cover_every_pair(nb):
    pairs, bmap = lyap.jacobi_schedule(nb)
    np_ = nb // 2
    seen = set()
    for t in range(nb):
        blocks = pairs[t].reshape(-1)
        assert sorted(blocks.tolist()) == list(range(nb))  # perfect matching
        for k in range(np_):
            i, j = int(pairs[t, k, 0]), int(pairs[t, k, 1])
            assert i < j
            assert bmap[t, i] == 2 * k and bmap[t, j] == 2 * k + 1
            pseudo = t % 2 == 0 and k == np_ - 1
            if pseudo:
                assert (i, j) == (t // 2, t // 2 + np_)
            else:
                assert (i + j) % nb == t
                assert (i, j) not in seen
                seen.add((i, j))
        if t % 2 == 1:
            assert all((int(a) + int(b)) % nb == t for a, b in pairs[t])
    assert seen == set(itertools.combinations(range(nb), 2))


@pytest.mark.parametrize("nb", [2, 4, 8, 12, 32, 64])
def test_first_two_rounds_cover_every_block(nb):
    pairs, _ = lyap.jacobi_schedule(nb)
    real = set()
    for t in (0, 1):
        for k, (i, j) in enumerate(pairs[t]):
            if not (t % 2 == 0 and k == nb // 2 - 1):
                real.update((int(i), int(j)))
    assert real == set(range(nb))


def _row_cyclic_pos(i, j, nb):
    # position of pair (i, j), i < j, in the row-cyclic sequence of one sweep
    return i * nb - i * (i + 1) // 2 + (j - i - 1)


@pytest.mark.parametrize("nb", [4, 6, 8, 16, 40])
def test_equivalent_to_row_cyclic(nb):
    """Over four sweeps of rounds, each block's pairs come in row-cyclic order and every
    row-cyclic sweep that lies wholly inside the window appears complete."""
    pairs, _ = lyap.jacobi_schedule(nb)
    np_ = nb // 2
    sweeps = 4
    events = []  # (absolute round, row-cyclic sweep, pair)
    for T in range(sweeps * nb):
        t = T % nb
        for k in range(np_):
            if t % 2 == 0 and k == np_ - 1:
                continue
            i, j = int(pairs[t, k, 0]), int(pairs[t, k, 1])
            s, rem = divmod(T - (i + j), nb)
            assert rem == 0  # round = i + j + s nb
            events.append((T, s, (i, j)))
    for b in range(nb):
        mine = [(T, s, p) for T, s, p in events if b in p]
        mine.sort()
        keys = [(s, _row_cyclic_pos(p[0], p[1], nb)) for _, s, p in mine]
        assert keys == sorted(keys)
        times = [T for T, _, _ in mine]
        assert len(set(times)) == len(times)  # a block is in one pair per round
    for s in range(0, sweeps - 2):
        got = sorted(p for _, ss, p in events if ss == s)
        assert got == sorted(itertools.combinations(range(nb), 2))


@pytest.mark.parametrize("nb", [0, 1, 3, 258, -2])
def test_bad_sizes_rejected(nb):
    with pytest.raises(_lib.LyapError) as e:
        lyap.jacobi_schedule(nb)
    assert e.value.status == "BADARG"
