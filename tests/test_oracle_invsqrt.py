"""Oracle inverse square root (coupled Newton-Schulz) against the eigendecomposition
and the closed-form residuals of the untruncated iteration."""
import math

import numpy as np
import pytest

import oracle as O
import synth


def _setup(s, rz):
    P6 = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    S = O.from_blocks(P6, s.b, s.S.rows, s.S.cols, s.S.blocks)
    PZ = O.create_pattern(s.positions, s.box, rz)
    return S, PZ


def _dense_powers(S):
    lam, V = np.linalg.eigh(S.to_dense())
    return lam, (V / np.sqrt(lam)) @ V.T, (V * np.sqrt(lam)) @ V.T


def test_untruncated_closed_form(si64):
    # With Z and Y on full patterns both are polynomials in A = alpha S, so
    # Z_k Y_k has the eigenvalues p_k of the scalar map p <- p (3 - p)^2 / 4 from
    # p_0 = alpha lambda: the residual is sqrt(sum (1 - p_k)^2), and the limits are
    # S^-1/2 and S^1/2.
    S, PZ = _setup(si64, 30.0)
    res = O.inverse_sqrt(S, PZ, max_iter=60, tol=1e-12)
    assert res.status == O.OK
    Sd = S.to_dense()
    a = 1.0 / np.abs(Sd).sum(1).max()
    assert res.alpha == pytest.approx(a, rel=1e-15)
    lam, Sm12, S12 = _dense_powers(S)
    p = a * lam
    for r in res.residuals:
        want = math.sqrt(np.sum((1.0 - p) ** 2))
        assert r == pytest.approx(want, rel=1e-8, abs=1e-12)
        p = p * (3.0 - p) ** 2 / 4.0
    np.testing.assert_allclose(res.Z.to_dense(), Sm12, atol=1e-12)
    np.testing.assert_allclose(res.Y.to_dense(), S12, atol=1e-12)
    np.testing.assert_allclose(res.Z.to_dense() @ Sd @ res.Z.to_dense(), np.eye(len(Sd)), atol=1e-11)


def test_fixed_iteration_count(si64):
    S, PZ = _setup(si64, 30.0)
    res = O.inverse_sqrt(S, PZ, max_iter=3, tol=0.0)
    assert res.iterations == 3 and res.status == O.OK and len(res.residuals) == 4


def test_truncated(si64):
    # Truncated at 6 A (the 64-atom cell is full from 9.41 A): symmetric iterates,
    # monotone residuals down to an accepted floor, and a result close to the
    # exact S^-1/2 on its pattern, closer at 8 A than at 6 A.
    errs = []
    for rz in (6.0, 8.0):
        S, PZ = _setup(si64, rz)
        res = O.inverse_sqrt(S, PZ, max_iter=100, tol=1e-12)
        assert res.status == O.OK
        assert all(b < a for a, b in zip(res.residuals, res.residuals[1:]))
        assert res.residuals[-1] <= 0.1 * math.sqrt(S.nrows)
        for M in (res.Z, res.Y):
            np.testing.assert_array_equal(M.blocks, O.transpose(M).blocks)
        _, Sm12, _ = _dense_powers(S)
        best = O.from_dense(PZ, S.b, Sm12)
        errs.append(np.linalg.norm(res.Z.blocks - best.blocks) / np.linalg.norm(best.blocks))
    assert errs[1] < errs[0] < 0.1


def test_indefinite_overlap_diverges():
    s = synth.make_system("bad", 2, 4, synth.SMALL_CUTOFFS, 2205, s_amp=3.0)
    S, PZ = _setup(s, 8.0)
    assert np.linalg.eigvalsh(S.to_dense()).min() < 0
    res = O.inverse_sqrt(S, PZ, max_iter=200, tol=1e-12)
    assert res.status == O.EDIVERGED


def test_nonfinite_input(si64):
    S, PZ = _setup(si64, 8.0)
    S.blocks[5, 1, 2] = np.nan
    res = O.inverse_sqrt(S, PZ, max_iter=5, tol=1e-12)
    assert res.status == O.ENONFINITE
