"""Oracle masked products and traces against dense numpy definitions."""
import numpy as np
import pytest

import oracle as O
import synth


def _mask(P):
    m = np.zeros((P.natoms, P.natoms))
    m[P.rows(), P.cols] = 1.0
    return m


def _rand(P, b, seed):
    return O.Matrix(P, b, synth.random_blocks(P.nnz, b, seed))


@pytest.fixture(scope="module")
def pats():
    s = synth.make_system("d", 2, 4, synth.SMALL_CUTOFFS, 3, displacement_sigma=0.1)
    return {r: O.create_pattern(s.positions, s.box, r) for r in (3.0, 5.0, 6.0, 8.0, 30.0)}


@pytest.mark.parametrize("ra,rb,rc", [(6, 6, 8), (8, 6, 5), (3, 8, 6), (30, 30, 30), (5, 3, 3)])
@pytest.mark.parametrize("b", [4, 9])
def test_product_vs_dense_masked(pats, ra, rb, rc, b):
    A, B = _rand(pats[ra], b, 1), _rand(pats[rb], b, 2)
    C = _rand(pats[rc], b, 3)
    C0 = C.to_dense()
    O.multiply_truncate(0.7, A, B, -1.3, C)
    M = np.kron(_mask(pats[rc]), np.ones((b, b)))
    want = 0.7 * (A.to_dense() @ B.to_dense()) * M - 1.3 * C0
    np.testing.assert_allclose(C.to_dense(), want, rtol=0, atol=1e-12)


def test_beta_zero_ignores_old_values(pats):
    A, B = _rand(pats[6], 4, 1), _rand(pats[6], 4, 2)
    C = O.Matrix(pats[8], 4, np.full((pats[8].nnz, 4, 4), np.nan))
    O.multiply_truncate(1.0, A, B, 0.0, C)
    assert np.isfinite(C.blocks).all()


def test_row_range(pats):
    A, B = _rand(pats[6], 4, 1), _rand(pats[6], 4, 2)
    C1 = O.product(A, B, pats[8])
    C2 = O.Matrix(pats[8], 4)
    O.multiply_truncate(1.0, A, B, 0.0, C2, 10, 30)
    r = pats[8].rows()
    sel = (r >= 10) & (r < 30)
    assert np.array_equal(C1.blocks[sel], C2.blocks[sel])
    assert not C2.blocks[~sel].any()


def test_count_triples_vs_boolean_products(pats):
    for ra, rb, rc in [(6, 6, 8), (8, 6, 5), (3, 8, 6)]:
        got = O.count_triples(pats[ra], pats[rb], pats[rc])
        want = ((_mask(pats[ra]) @ _mask(pats[rb])) * _mask(pats[rc])).sum(1)
        assert np.array_equal(got, want.astype(np.int64))


def test_count_triples_4096_w_class():
    # the 16 A x 16 A -> 16 A product at 4096 atoms: 398 k-terms per output block on average
    pos, box, _ = synth.diamond_positions((8, 8, 8))
    P = O.create_pattern(pos, box, 16.0)
    t = O.count_triples(P, P, P)
    m = np.zeros((4096, 4096), np.float32)
    m[P.rows(), P.cols] = 1
    want = ((m @ m) * m).sum(1)
    assert np.array_equal(t, want.astype(np.int64))
    assert np.all(t == t[0])          # perfect crystal: every row alike
    assert round(t[0] / 849) == 398


@pytest.mark.parametrize("ra,rb", [(6, 6), (6, 8), (3, 30), (8, 5)])
def test_trace_vs_dense(pats, ra, rb):
    A, B = _rand(pats[ra], 4, 5), _rand(pats[rb], 4, 6)
    want = np.trace(A.to_dense() @ B.to_dense())
    assert abs(O.trace_product(A, B) - want) <= 1e-12 * max(1.0, abs(want))


def test_helpers(pats):
    A = _rand(pats[6], 4, 9)
    D = A.to_dense()
    np.testing.assert_array_equal(O.transpose(A).to_dense(), D.T)
    np.testing.assert_allclose(O.symmetrize(A).to_dense(), 0.5 * (D + D.T), atol=0)
    assert O.trace(A) == pytest.approx(np.trace(D), abs=1e-13)
    B = _rand(pats[6], 4, 10)
    assert O.dot(A, B) == pytest.approx(np.sum(D * B.to_dense()), abs=1e-12)
    m = O.mask_copy(A, pats[3])
    np.testing.assert_array_equal(m.to_dense(), D * np.kron(_mask(pats[3]), np.ones((4, 4))))
