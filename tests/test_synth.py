"""Generator checks: shapes, symmetry, SPD overlap, gapped (H, S) with 2N occupied states."""
import numpy as np
import pytest
import scipy.linalg as sl

import synth


@pytest.mark.parametrize("b", [4, 9])
def test_small_system_spectrum(b):
    s = synth.make_system("t", 2, b, synth.SMALL_CUTOFFS, 2205)
    n = s.natoms
    assert n == 64 and s.n_electrons == 256
    S, H = s.S.to_dense(n), s.H.to_dense(n)
    assert np.array_equal(S, S.T) and np.array_equal(H, H.T)
    ev = np.linalg.eigvalsh(S)
    assert 0.3 < ev.min() and ev.max() < 1.8
    w = sl.eigh(H, S, eigvals_only=True)
    # exactly 2N states below the gap at zero energy (spin-paired, 4 electrons per atom)
    assert (w < 0).sum() == 2 * n
    assert w[w < 0].max() < -0.1 and w[w > 0].min() > 0.1


def test_seeded_and_order_independent():
    a = synth.make_system("t", 2, 4, synth.SMALL_CUTOFFS, 7)
    b = synth.make_system("t", 2, 4, synth.SMALL_CUTOFFS, 7)
    c = synth.make_system("t", 2, 4, synth.SMALL_CUTOFFS, 8)
    assert np.array_equal(a.S.blocks, b.S.blocks) and np.array_equal(a.H.blocks, b.H.blocks)
    assert not np.allclose(a.S.blocks, c.S.blocks)


def test_folding_of_images():
    # 64 atoms in a 10.86 A box: some pairs have two images within 6 A; folding sums them
    s = synth.si64_b4()
    i, j, sh, d = synth.image_pairs(s.positions, s.box, 6.0)
    key = i * 64 + j
    _, counts = np.unique(key, return_counts=True)
    assert counts.max() == 2
    assert len(s.S.rows) == 64 * 44


def test_counter_uniform_range():
    u = synth.counter_uniform(1, 2, np.arange(100000))
    assert u.min() >= 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 0.01


def test_smooth_derivative_blocks_match_finite_differences():
    # dS, dH hold d(block ij)/dR_j (and -d/dR_i); central differences of the
    # generator itself, moving one atom, agree to rounding.
    kw = dict(displacement_sigma=0.05, smooth=True)
    s = synth.make_system("f", 2, 4, synth.SMALL_CUTOFFS, 11, derivatives=True, **kw)
    J, h = 5, 1e-5
    for c in range(3):
        e = np.zeros((s.natoms, 3))
        e[J, c] = h
        p = synth.make_system("f", 2, 4, synth.SMALL_CUTOFFS, 11, extra_displacement=e, **kw)
        m = synth.make_system("f", 2, 4, synth.SMALL_CUTOFFS, 11, extra_displacement=-e, **kw)
        for name in ("S", "H"):
            D = getattr(s, "d" + name)[c]
            assert np.array_equal(D.rows, getattr(s, name).rows) and np.array_equal(D.cols, getattr(s, name).cols)
            fd = (getattr(p, name).blocks - getattr(m, name).blocks) / (2 * h)
            want = np.zeros_like(fd)
            col, row = (D.cols == J) & (D.rows != J), (D.rows == J) & (D.cols != J)
            want[col], want[row] = D.blocks[col], -D.blocks[row]
            assert np.abs(fd - want).max() < 1e-9 * max(1.0, np.abs(want).max())
