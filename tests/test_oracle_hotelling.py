"""Oracle Hotelling iteration against the dense inverse and its closed-form residuals."""
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


def test_untruncated_closed_form(si64):
    # With Z on the full pattern, I - Z_n S = (I - a S)^(2^n), so the residual at
    # step n is sqrt(sum_k (1 - a lambda_k)^(2^(n+1))) and the limit is S^-1.
    S, PZ = _setup(si64, 30.0)
    res = O.hotelling_inverse(S, PZ, max_iter=50, tol=1e-12)
    assert res.status == O.OK
    lam = np.linalg.eigvalsh(S.to_dense())
    a = res.alpha
    assert a == pytest.approx(1.0 / np.abs(S.to_dense()).sum(1).max(), rel=1e-15)
    for n, r in enumerate(res.residuals):
        want = math.sqrt(np.sum((1.0 - a * lam) ** (2 ** (n + 1))))
        assert r == pytest.approx(want, rel=1e-8, abs=1e-13)
    np.testing.assert_allclose(res.Z.to_dense(), np.linalg.inv(S.to_dense()), atol=1e-12)


def test_fixed_iteration_count(si64):
    S, PZ = _setup(si64, 30.0)
    res = O.hotelling_inverse(S, PZ, max_iter=3, tol=0.0)
    assert res.iterations == 3 and res.status == O.OK and len(res.residuals) == 4


@pytest.mark.slow
def test_truncated_plateau_512():
    # Truncated at 8 A the iteration stalls near ||I - mask(S^-1) S||_F, the residual
    # of the best-truncated exact inverse.
    s = synth.make_system("t", 4, 4, synth.SMALL_CUTOFFS, 2205)
    S, PZ = _setup(s, 8.0)
    res = O.hotelling_inverse(S, PZ, max_iter=100, tol=1e-12)
    assert res.status == O.OK
    Sd = S.to_dense()
    Zt = O.from_dense(PZ, 4, np.linalg.inv(Sd)).to_dense()
    best = np.linalg.norm(np.eye(len(Sd)) - Zt @ Sd)
    assert abs(res.residuals[-1] - best) / best < 0.05
    # near a fixed point of the truncated map
    Z = res.Z
    step = O.symmetrize(O.Matrix(PZ, 4, 2 * Z.blocks - O.product(O.product(Z, S, O.create_pattern(s.positions, s.box, 14.0)), Z, PZ).blocks))
    assert np.linalg.norm(step.blocks - Z.blocks) / np.linalg.norm(Z.blocks) < 0.05
    # monotone residuals
    assert all(b < a for a, b in zip(res.residuals, res.residuals[1:]))


def test_indefinite_overlap_diverges():
    s = synth.make_system("bad", 2, 4, synth.SMALL_CUTOFFS, 2205, s_amp=3.0)
    S, PZ = _setup(s, 8.0)
    assert np.linalg.eigvalsh(S.to_dense()).min() < 0
    res = O.hotelling_inverse(S, PZ, max_iter=200, tol=1e-12)
    assert res.status == O.EDIVERGED


def test_nonfinite_input(si64):
    S, PZ = _setup(si64, 8.0)
    S.blocks[5, 1, 2] = np.nan
    res = O.hotelling_inverse(S, PZ, max_iter=5, tol=1e-12)
    assert res.status == O.ENONFINITE
