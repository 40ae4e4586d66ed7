"""Oracle contraction to support functions: selection, congruence symmetry, rotation
invariance of the ground-state energy and the Rayleigh-Ritz bound."""
import numpy as np
import scipy.linalg as sl

import oracle as O
import synth


def _system(rs=10.0):
    s = synth.make_system("c", 2, 9, {"S": rs, "H": rs, "L": rs, "Z": rs}, 5)
    P = O.create_pattern(s.positions, s.box, rs)
    return s, O.from_blocks(P, 9, s.S.rows, s.S.cols, s.S.blocks), O.from_blocks(P, 9, s.H.rows, s.H.cols, s.H.blocks)


def _onsite_coef(H, bc):
    d = H.pattern.diag_slots()
    return np.stack([np.linalg.eigh(H.blocks[k])[1][:, :bc] for k in d])


def _band_energy(S, H, n_occ):
    w = sl.eigh(H.to_dense(), S.to_dense(), eigvals_only=True)
    return 2.0 * w[:n_occ].sum()


def test_selection_coefficients_pick_sub_blocks():
    s, S, H = _system(6.0)
    coef = np.broadcast_to(np.eye(9)[:, :4], (s.natoms, 9, 4))
    Sc = O.contract(S, coef)
    np.testing.assert_array_equal(Sc.blocks, S.blocks[:, :4, :4])


def test_contracted_matrices_stay_symmetric():
    # a wrong side (C_i vs C_j, or a missing transpose) breaks M'_ji = M'_ij^T
    s, S, H = _system(6.0)
    coef = np.random.default_rng(1).normal(size=(s.natoms, 9, 4))
    for M in (S, H):
        Mc = O.contract(M, coef)
        np.testing.assert_allclose(Mc.blocks, O.transpose(Mc).blocks, atol=1e-14)


def test_energy_invariant_under_support_rotations_and_bounded():
    # rotating each atom's support functions is a congruence of (H', S'): the occupied
    # eigenvalues do not change; the contracted energy bounds the full one from above
    s, S, H = _system()
    n_occ = int(s.n_electrons // 2)
    coef = _onsite_coef(H, 4)
    E1 = _band_energy(O.contract(S, coef), O.contract(H, coef), n_occ)
    rot = np.stack([np.linalg.qr(np.random.default_rng(k).normal(size=(4, 4)))[0] for k in range(s.natoms)])
    E2 = _band_energy(O.contract(S, coef @ rot), O.contract(H, coef @ rot), n_occ)
    Efull = _band_energy(S, H, n_occ)
    assert abs(E1 - E2) < 1e-10 * abs(E1)
    assert E1 >= Efull - 1e-10 and E1 - Efull < 0.05 * abs(Efull)
