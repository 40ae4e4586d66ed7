"""Oracle forces from the converged density matrix against central differences of
the converged energy (the generator's geometry-smooth S and H), and translation
invariance."""
import numpy as np
import pytest

import oracle as O
import synth

KW = dict(displacement_sigma=0.05, smooth=True)


def _solve(s, tol=1e-13):
    P6 = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    S = O.from_blocks(P6, s.b, s.S.rows, s.S.cols, s.S.blocks)
    H = O.from_blocks(P6, s.b, s.H.rows, s.H.cols, s.H.blocks)
    Z = O.hotelling_inverse(S, O.create_pattern(s.positions, s.box, s.cutoffs["Z"]), max_iter=100).Z
    st = O.lnv_init(S, H, Z, O.create_pattern(s.positions, s.box, s.cutoffs["L"]), s.n_electrons, tol_E=tol)
    out = O.lnv_solve(st, [(O.F64, 1000, tol, False)])
    assert out["converged"] and out["status"] == O.OK
    return st, out["E"], P6


@pytest.fixture(scope="module")
def converged():
    s = synth.make_system("f", 2, 4, synth.SMALL_CUTOFFS, 11, derivatives=True, **KW)
    st, E, P6 = _solve(s)
    dS = [O.from_blocks(P6, s.b, d.rows, d.cols, d.blocks) for d in s.dS]
    dH = [O.from_blocks(P6, s.b, d.rows, d.cols, d.blocks) for d in s.dH]
    return s, st, E, O.lnv_forces(st, dS, dH)


def test_forces_sum_to_zero(converged):
    # every pair term enters the rows of both atoms with opposite signs
    _, _, _, F = converged
    assert np.abs(F).max() > 1e-3
    assert np.abs(F.sum(axis=0)).max() < 1e-10 * np.abs(F).max()


@pytest.mark.parametrize("atom,c", [(5, 1), (17, 0), (40, 2)])
def test_forces_match_energy_differences(converged, atom, c):
    s, _, _, F = converged
    h = 1e-4
    E = []
    for sign in (1.0, -1.0):
        e = np.zeros((s.natoms, 3))
        e[atom, c] = sign * h
        E.append(_solve(synth.make_system("f", 2, 4, synth.SMALL_CUTOFFS, 11, extra_displacement=e, **KW))[1])
    fd = -(E[0] - E[1]) / (2 * h)
    assert F[atom, c] == pytest.approx(fd, rel=1e-5, abs=1e-8)
