"""Oracle preconditioner M(G) and chemical potential mu against closed forms.

M(G) = sym(mask_L((Z G) Z)) is the S^-1-contravariant form of an LNV gradient;
mu = <G_N, M(G_E)> / <G_N, M(G_N)> is the canonical chemical potential.  Pins:

* full cutoffs, Z = S^-1 exactly: M(G) is the dense S^-1 G S^-1;
* truncated cutoffs: M(G) is mask_L of the dense product Z G Z, i.e. the
  intermediate Z G must be held exactly (on P(r_Z + r_L)), not cut to P_L;
* a spectral L = V diag(lam) V^T built from the generalised eigenvectors of
  (H, S) (V^T S V = I, V^T H V = diag(eps)): the gradients are diagonal in that
  basis, dE/dlam_n = g_n eps_n and dN/dlam_n = g_n with g_n = 12 lam_n (1 - lam_n),
  so with M = S^-1 (.) S^-1 the formula gives mu = sum g_n^2 eps_n / sum g_n^2.

Each pin is shown to catch a plausible mistake planted in the oracle (the
intermediate Z G cut to P_L, one Z factor dropped, mu with the wrong sign).
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
import synth


def _full_cutoff_state(seed=11):
    s = synth.si64_b4()
    P = O.create_pattern(s.positions, s.box, 30.0)         # every pair of the 64-atom cell
    P6 = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    S = O.from_blocks(P6, 4, s.S.rows, s.S.cols, s.S.blocks)
    H = O.from_blocks(P6, 4, s.H.rows, s.H.cols, s.H.blocks)
    Sd, Hd = S.to_dense(), H.to_dense()
    Sinv = np.linalg.inv(Sd)
    Z = O.from_dense(P, 4, 0.5 * (Sinv + Sinv.T))
    eps, V = sl.eigh(Hd, Sd)
    rng = np.random.default_rng(seed)
    lam = np.where(eps < 0, rng.uniform(0.6, 0.97, eps.size), rng.uniform(0.03, 0.4, eps.size))
    Ld = (V * lam) @ V.T
    L = O.from_dense(P, 4, 0.5 * (Ld + Ld.T))
    st = O.lnv_init(S, H, Z, P, s.n_electrons, L0=L)
    return st, Sinv, eps, lam


def _truncated_state():
    s = synth.make_system("pre512", 4, 4, synth.BIG_CUTOFFS, 17, displacement_sigma=0.05)
    P6 = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    S = O.from_blocks(P6, 4, s.S.rows, s.S.cols, s.S.blocks)
    H = O.from_blocks(P6, 4, s.H.rows, s.H.cols, s.H.blocks)
    PZ = O.create_pattern(s.positions, s.box, s.cutoffs["Z"])
    Z = O.hotelling_inverse(S, PZ, max_iter=100, tol=1e-12).Z
    PL = O.create_pattern(s.positions, s.box, s.cutoffs["L"])
    st = O.lnv_init(S, H, Z, PL, s.n_electrons)
    return st


def _random_symmetric(P, b, seed):
    return O.symmetrize(O.Matrix(P, b, synth.random_blocks(P.nnz, b, seed)))


def _dense_mask(P, b, D):
    return O.from_dense(P, b, D)


def _err_full(st, Sinv, G):
    M = O._precondition(st, G).to_dense()
    ref = Sinv @ G.to_dense() @ Sinv
    return np.abs(M - ref).max() / np.abs(ref).max()


def _err_truncated(st, G):
    M = O._precondition(st, G)
    Zd = st.Z.to_dense()
    ref = _dense_mask(st.L.pattern, st.L.b, Zd @ G.to_dense() @ Zd)
    return np.abs(M.blocks - ref.blocks).max() / np.abs(ref.blocks).max()


def _mu_closed_form(eps, lam):
    g = 12.0 * lam * (1.0 - lam)
    return float(np.sum(g * g * eps) / np.sum(g * g))


# ---- planted mistakes (each must make at least one pin fail) ------------------
def _zg_cut_to_pl(st, G):
    ZG = O.product(st.Z, G, st.L.pattern, st.prec)
    return O.symmetrize(O.product(ZG, st.Z, st.L.pattern, st.prec))


def _one_z_dropped(st, G):
    return O.symmetrize(O.product(st.Z, G, st.L.pattern, st.prec))


# ------------------------------------------------------------------------------
def test_precondition_full_cutoff_is_dense_sandwich():
    st, Sinv, _, _ = _full_cutoff_state()
    G = _random_symmetric(st.L.pattern, 4, 3)
    assert _err_full(st, Sinv, G) < 1e-12


def test_precondition_truncated_is_masked_dense_product():
    st = _truncated_state()
    P = st.L.pattern
    assert P.nnz < P.natoms ** 2 // 2          # L genuinely truncated
    assert st.PZG.nnz > P.nnz                   # Z G held on the wider pattern
    G = _random_symmetric(P, 4, 5)
    assert _err_truncated(st, G) < 1e-12


def test_mu_equals_spectral_weighted_mean():
    st, _, eps, lam = _full_cutoff_state()
    mu = O.lnv_chemical_potential(st)
    ref = _mu_closed_form(eps, lam)
    assert abs(mu - ref) <= 1e-10 * abs(ref)
    # the same value is what an LNV step uses (canonical mode)
    r = O.lnv_step(st)
    assert abs(r.mu - ref) <= 1e-10 * abs(ref)


def test_pins_catch_planted_mistakes(monkeypatch):
    # intermediate Z G cut to P_L: the truncated pin fails
    st = _truncated_state()
    G = _random_symmetric(st.L.pattern, 4, 5)
    monkeypatch.setattr(O, "_precondition", _zg_cut_to_pl)
    assert _err_truncated(st, G) > 1e-6
    # one Z factor dropped: the full-cutoff pin and the mu pin fail
    stf, Sinv, eps, lam = _full_cutoff_state()
    Gf = _random_symmetric(stf.L.pattern, 4, 3)
    monkeypatch.setattr(O, "_precondition", _one_z_dropped)
    assert _err_full(stf, Sinv, Gf) > 1e-3
    ref = _mu_closed_form(eps, lam)
    assert abs(O.lnv_chemical_potential(stf) - ref) > 1e-6 * abs(ref)
    monkeypatch.undo()
    # mu with the wrong sign
    mu = O.lnv_chemical_potential(stf)
    assert abs(-mu - ref) > 1e-3 * abs(ref)
