"""Oracle patterns against textbook shells, exact lattice counting and an independent brute force."""
import os

import numpy as np
import pytest

import oracle as O
import synth


def diamond_shell_count(r_over_quarter_a: float) -> int:
    """Diamond lattice points within r of an atom, counted exactly in units of a/4.

    In those units the lattice is the integer points whose coordinates are all
    even with x+y+z = 0 (mod 4), or all odd with x+y+z = 3 (mod 4).
    """
    m = int(np.ceil(r_over_quarter_a)) + 1
    g = np.arange(-m, m + 1)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    even = (x % 2 == 0) & (y % 2 == 0) & (z % 2 == 0) & ((x + y + z) % 4 == 0)
    odd = (x % 2 == 1) & (y % 2 == 1) & (z % 2 == 1) & ((x + y + z) % 4 == 3)
    d2 = x * x + y * y + z * z
    return int(((even | odd) & (d2 < r_over_quarter_a ** 2)).sum())


def textbook_shells():
    """(squared distance in (a/4)^2, shell size, cumulative count) from tests/golden."""
    path = os.path.join(os.path.dirname(__file__), "golden", "diamond_shells.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    return [tuple(int(v) for v in r) for r in rows]


def test_shell_count_helper_textbook_shells():
    # the first coordination shells of diamond, counted just outside each shell
    shells = textbook_shells()
    assert [s[1] for s in shells] == [4, 12, 12, 6] and shells[-1][2] == 35
    for d2, size, cum in shells:
        assert diamond_shell_count(np.sqrt(d2) + 0.05) == cum
        assert diamond_shell_count(np.sqrt(d2) - 0.05) == cum - size


def test_oracle_rows_match_textbook_shells():
    # the oracle's pattern on a periodic 4096-atom crystal, cut just outside each shell
    pos, box, _ = synth.diamond_positions((8, 8, 8))
    q = synth.A_SI / 4
    for d2, size, cum in textbook_shells():
        P = O.create_pattern(pos, box, (np.sqrt(d2) + 0.05) * q)
        assert np.all(np.diff(P.rowptr) == cum), d2


@pytest.mark.parametrize("r", [6.0, 8.0, 10.0, 16.0])
def test_rows_match_lattice_count_4096(r):
    pos, box, _ = synth.diamond_positions((8, 8, 8))
    P = O.create_pattern(pos, box, r)
    expect = diamond_shell_count(r / (synth.A_SI / 4))
    assert np.all(np.diff(P.rowptr) == expect)


def test_small_box_counts():
    s = synth.si64_b4()
    for r, want in [(6.0, 44), (8.0, 63), (10.0, 64), (30.0, 64)]:
        P = O.create_pattern(s.positions, s.box, r)
        assert np.all(np.diff(P.rowptr) == want), r


def test_brute_force_all_images_displaced():
    s = synth.make_system("d", 2, 4, synth.SMALL_CUTOFFS, 11, displacement_sigma=0.2)
    pos, box = s.positions, s.box
    for r in [4.0, 6.0, 7.3]:
        P = O.create_pattern(pos, box, r)
        shifts = np.stack(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1], indexing="ij"), -1).reshape(-1, 3)
        dv = pos[None, :, None, :] + shifts[None, None] * box - pos[:, None, None, :]
        dmin = np.sqrt((dv ** 2).sum(-1)).min(-1)
        want = (dmin < r) | np.eye(len(pos), dtype=bool)
        got = np.zeros_like(want)
        got[P.rows(), P.cols] = True
        assert np.array_equal(got, want)
        assert np.array_equal(got, got.T)
        for i in range(len(pos)):
            c = P.cols[P.rowptr[i]:P.rowptr[i + 1]]
            assert np.all(np.diff(c) > 0)
