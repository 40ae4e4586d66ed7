"""The stored oracle solves (tests/golden/lnv_<case>.json) against facts fixed outside the oracle.

The GPU golden test trusts these files; here they are checked on the CPU without re-running
the oracle (the 4096-atom solve takes hours):

* the seeded system they were written for is the one the input generator builds today: the
  Hotelling start Z0 = I / rho (rho the Gershgorin bound, from the generator's S blocks in plain
  numpy) and its residual ||I - S / rho||_F equal the stored alpha and first residual;
* Hotelling residuals fall at every stored update and stop at the truncation floor
  (at most 0.1 sqrt(N_b));
* the LNV energy falls at every iteration, the last |dE| is below the tolerance, the electron
  count ends at N_e, and the stored final energy is the last iteration's;
* the record is complete: a row norm per atom for S^-1 and L, 64 samples of each with the
  orbital count's block size.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = ["si512_b9_disp", "si4096_b9"]


def system(case):
    if case == "si4096_b9":
        return synth.si4096_b9()
    return synth.make_system("si512_b9_disp", 4, 9, synth.BIG_CUTOFFS, 7, displacement_sigma=0.05)


def load(case):
    path = os.path.join(HERE, "golden", f"lnv_{case}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not present")
    with open(path) as f:
        return json.load(f)


def gershgorin_and_start_residual(s):
    """rho = max over scalar rows of sum_j |S_ij|, and ||I - S / rho||_F, from the block list."""
    b, n = s.b, s.natoms
    rows, cols, blocks = np.asarray(s.S.rows), np.asarray(s.S.cols), np.asarray(s.S.blocks)
    rowsum = np.zeros(n * b)
    np.add.at(rowsum, (rows[:, None] * b + np.arange(b)[None, :]).ravel(), np.abs(blocks).sum(axis=2).ravel())
    rho = rowsum.max()
    R = -blocks / rho
    diag = rows == cols
    R[diag] += np.eye(b)
    return rho, math.sqrt(float(np.sum(R * R)))


@pytest.mark.parametrize("case", CASES)
def test_stored_solve_belongs_to_todays_system(case):
    g = load(case)
    s = system(case)
    gen = g["generator"]
    assert gen["natoms"] == s.natoms and gen["b"] == s.b and gen["seed"] == s.seed
    assert gen["n_electrons"] == s.n_electrons and gen["cutoffs_A"] == s.cutoffs
    # every (i, j) pair appears once in the generator's S
    assert len(set(zip(np.asarray(s.S.rows).tolist(), np.asarray(s.S.cols).tolist()))) == len(s.S.rows)
    rho, r0 = gershgorin_and_start_residual(s)
    h = g["hotelling"]
    assert h["alpha"] == pytest.approx(1.0 / rho, rel=1e-14)
    assert h["residuals"][0] == pytest.approx(r0, rel=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_stored_solve_is_a_converged_descent(case):
    g = load(case)
    gen, h, lnv = g["generator"], g["hotelling"], g["lnv"]
    nb = gen["natoms"] * gen["b"]
    res = np.array(h["residuals"])
    assert h["status"] == 0 and len(res) == h["iterations"] + 1
    assert np.all(np.diff(res) < 0)
    assert res[-1] <= 0.1 * math.sqrt(nb)
    it = lnv["iterations"]
    E = np.array([x["E"] for x in it])
    assert lnv["converged"] and 1 < len(it) <= lnv["max_iter"]
    assert np.all(np.diff(E) < 0)
    assert abs(it[-1]["dE"]) < lnv["tol_E"] and all(abs(x["dE"]) >= lnv["tol_E"] for x in it[1:-1])
    assert abs(it[-1]["N"] - gen["n_electrons"]) <= 1e-9 * gen["n_electrons"]
    assert lnv["E_final"] == it[-1]["E"]
    for k in ("alpha", "mu", "Omega"):
        assert all(math.isfinite(x[k]) for x in it)
    assert all(x["alpha"] > 0 for x in it)
    if "idempotency_error" in lnv:
        assert 0 < lnv["idempotency_error"] < 1e-3


@pytest.mark.parametrize("case", CASES)
def test_stored_solve_record_is_complete(case):
    g = load(case)
    n, b = g["generator"]["natoms"], g["generator"]["b"]
    for m in ("Z", "L"):
        norms = np.array(g[f"{m}_row_norms"])
        assert norms.shape == (n,) and np.all(norms > 0)
        smp = g[f"{m}_samples"]
        assert len(smp["rows"]) == len(smp["cols"]) == len(smp["blocks"]) == 64
        assert all(len(blk) == b * b for blk in smp["blocks"])
        assert all(0 <= i < n and 0 <= j < n for i, j in zip(smp["rows"], smp["cols"]))
    assert g["L_norm"] == pytest.approx(math.sqrt(float(np.sum(np.square(g["L_row_norms"])))), rel=1e-12)
