"""Oracle LNV minimisation against dense definitions, finite differences and eigenvalues."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
import synth


def _system(s, rl=None, rz=None, hot_iter=100):
    rl = s.cutoffs["L"] if rl is None else rl
    rz = s.cutoffs["Z"] if rz is None else rz
    P6 = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    S = O.from_blocks(P6, s.b, s.S.rows, s.S.cols, s.S.blocks)
    H = O.from_blocks(P6, s.b, s.H.rows, s.H.cols, s.H.blocks)
    PZ = O.create_pattern(s.positions, s.box, rz)
    Z = O.hotelling_inverse(S, PZ, max_iter=hot_iter, tol=1e-12).Z
    PL = O.create_pattern(s.positions, s.box, rl)
    return S, H, Z, PL


def _dense_E_N(L, S, H):
    K = 3 * L @ S @ L - 2 * L @ S @ L @ S @ L
    return 2 * np.trace(K @ H), 2 * np.trace(K @ S)


def _sym_direction(P, b, seed):
    D = O.Matrix(P, b, synth.random_blocks(P.nnz, b, seed, scale=0.01))
    return O.symmetrize(D)


def test_energy_terms_vs_dense(si64):
    S, H, Z, PL = _system(si64)
    st = O.lnv_init(S, H, Z, PL, si64.n_electrons)
    st.L = O.Matrix(PL, 4, st.L.blocks + _sym_direction(PL, 4, 3).blocks)
    *_, E, N = O.lnv_energy_terms(st)
    Ed, Nd = _dense_E_N(st.L.to_dense(), S.to_dense(), H.to_dense())
    assert E == pytest.approx(Ed, rel=1e-12) and N == pytest.approx(Nd, rel=1e-12)


def test_initial_guess_electron_count(si64):
    S, H, Z, PL = _system(si64)
    st = O.lnv_init(S, H, Z, PL, si64.n_electrons)
    _, Nd = _dense_E_N(st.L.to_dense(), S.to_dense(), H.to_dense())
    assert Nd == pytest.approx(si64.n_electrons, rel=1e-12)


def test_initial_scale_closed_form():
    # with Z = S^-1 exactly, t2 = t3 = N_b and c solves 3c^2 - 2c^3 = N_e / (2 N_b)
    assert O.lnv_initial_scale(256, 256.0, 256.0, 256.0) == pytest.approx(0.5, abs=1e-15)
    c = O.lnv_initial_scale(576, 256.0, 576.0, 576.0)
    assert 3 * c * c - 2 * c ** 3 == pytest.approx(256.0 / 1152.0, rel=1e-14)
    assert 0.30 < c < 0.31


@pytest.mark.parametrize("which", ["E", "N"])
def test_gradient_vs_finite_differences(si64, which):
    S, H, Z, PL = _system(si64)
    st = O.lnv_init(S, H, Z, PL, si64.n_electrons)
    X, Y, W, U, E, N = O.lnv_energy_terms(st)
    GE, GN = O.lnv_gradients(st, X, W, U)
    G = GE if which == "E" else GN
    D = _sym_direction(PL, 4, 8)
    L0 = st.L.blocks.copy()

    def f(eps):
        st.L = O.Matrix(PL, 4, L0 + eps * D.blocks)
        r = O.lnv_energy_terms(st)
        return r[4] if which == "E" else r[5]

    h = 0.5
    # f is a cubic polynomial in eps, so this 4-point stencil is exact up to rounding
    fd = (8 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12 * h)
    assert O.dot(G, D) == pytest.approx(fd, rel=1e-9)


def test_line_search_cubic_and_c1(si64):
    S, H, Z, PL = _system(si64)
    st = O.lnv_init(S, H, Z, PL, si64.n_electrons)
    for _ in range(3):
        O.lnv_step(st)
    L0 = st.L.to_dense()
    # reproduce the step by hand to get D, then check Omega(alpha) densely
    X, Y, W, U, E, N = O.lnv_energy_terms(st)
    res = O.lnv_step(st)
    c = res.c
    D = st.D_prev.to_dense()
    Sd, Hd = S.to_dense(), H.to_dense()
    for a in [-0.3, 0.2, 0.7, 1.1]:
        Ea, Na = _dense_E_N(L0 + a * D, Sd, Hd)
        Om = Ea - res.mu * Na
        poly = c[0] + a * (c[1] + a * (c[2] + a * c[3]))
        assert Om == pytest.approx(poly, rel=1e-11)
    assert c[1] < 0
    assert c[1] == pytest.approx(O.dot(st.g_prev, st.D_prev), rel=1e-9)


def test_full_cutoff_matches_eigenvalue_sum(si64):
    # cutoffs covering the whole cell: LNV reduces to exact minimisation, so E is
    # twice the sum of the 2N lowest generalised eigenvalues and K is idempotent.
    S, H, Z, PL = _system(si64, rl=30.0, rz=30.0)
    st = O.lnv_init(S, H, Z, PL, si64.n_electrons, tol_E=1e-11)
    for _ in range(100):
        r = O.lnv_step(st)
        if r.converged:
            break
    Sd, Hd = S.to_dense(), H.to_dense()
    w = sl.eigh(Hd, Sd, eigvals_only=True)
    assert r.E == pytest.approx(2 * w[:128].sum(), abs=1e-7)
    L = st.L.to_dense()
    K = 3 * L @ Sd @ L - 2 * L @ Sd @ L @ Sd @ L
    assert np.linalg.norm(K @ Sd @ K - K) / np.linalg.norm(K) < 1e-4
    assert 2 * np.trace(K @ Sd) == pytest.approx(si64.n_electrons, rel=1e-9)


def test_truncated_energy_is_variational(si64):
    S, H, Z, PL = _system(si64, rl=6.0)
    st = O.lnv_init(S, H, Z, PL, si64.n_electrons)
    for _ in range(60):
        r = O.lnv_step(st)
        if r.converged:
            break
    w = sl.eigh(H.to_dense(), S.to_dense(), eigvals_only=True)
    assert r.E > 2 * w[:128].sum()


@pytest.mark.parametrize("b", [4, 9])
def test_bond_projector_closed_form(b):
    # S = I and H = bonds only (+ d levels): K is the bond projector, E = -4 N t exactly
    s = synth.make_system("bond", 2, b, synth.SMALL_CUTOFFS, 5, s_amp=0.0, h_random=False)
    S, H, Z, PL = _system(s)
    st = O.lnv_init(S, H, Z, PL, s.n_electrons, tol_E=1e-12)
    for _ in range(100):
        r = O.lnv_step(st)
        if r.converged:
            break
    assert r.E == pytest.approx(-4 * 64 * synth.T_BOND, abs=1e-9)
    assert r.N == pytest.approx(256.0, abs=1e-9)


def test_grand_mode_monotone(si64):
    S, H, Z, PL = _system(si64)
    st = O.lnv_init(S, H, Z, PL, si64.n_electrons, mode=O.GRAND, mu=0.0)
    om = [O.lnv_step(st).Omega for _ in range(12)]
    assert all(b < a for a, b in zip(om, om[1:]))


def test_runaway_detected(si64):
    # L = 2 Z puts the LS spectrum near 2, outside the basin (-1/2, 3/2): with mu far
    # below the spectrum the cubic has no minimum
    S, H, Z, PL = _system(si64)
    L0 = O.Matrix(Z.pattern, 4, 2.0 * Z.blocks)
    st = O.lnv_init(S, H, Z, PL, si64.n_electrons, mode=O.GRAND, mu=-10.0, L0=L0)
    r = O.lnv_step(st)
    assert r.status == O.ERUNAWAY
