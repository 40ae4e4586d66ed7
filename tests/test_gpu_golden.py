"""GPU Hotelling + LNV solves against stored FP64 oracle solves of the same seeded systems.

The stored values (tests/golden/lnv_<case>.json) were written by
tests/golden/make_lnv_golden.py, which calls only the oracle and the input
generator.  Cases:

* si512_b9_disp: 512 displaced atoms, 9 orbitals, S/H on 6 A, S^-1 on 8 A, L on
  10 A -- the L, S^-1 and S patterns and the derived ones are truncated, so the
  wide intermediate patterns, transposed plans and fused trace sets are all
  exercised against the oracle;
* si4096_b9: the 4096-atom, 9-orbital benchmark system, solved to |dE| < 1e-8 Ha
  in the launch configuration the benchmark times.

Bars: Hotelling residuals and the update count equal to the oracle's (residuals
within 1e-10 relative), sampled S^-1 blocks and every S^-1 block-row norm within
1e-10 of the result scale; LNV E and N within 1e-10 relative at every iteration,
alpha within 1e-6 for the first 6 iterations (later alpha is a ratio of traces
that cancel to rounding level), the same iteration count, sampled L blocks with
||dL|| / ||L|| <= 1e-8 and block-row norms within 1e-8; where stored, the
idempotency error ||KS KS - KS|| / ||KS|| of the converged L within 1e-8 relative.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def golden(case):
    path = os.path.join(HERE, "golden", f"lnv_{case}.json")
    if not os.path.exists(path):
        pytest.skip(f"stored oracle solve {path} not present")
    with open(path) as f:
        return json.load(f)


def system(case):
    if case == "si4096_b9":
        return synth.si4096_b9()
    if case == "si512_b9_disp":
        return synth.make_system("si512_b9_disp", 4, 9, synth.BIG_CUTOFFS, 7, displacement_sigma=0.05)
    raise ValueError(case)


@pytest.fixture(scope="module")
def bsm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_08941_amd as bsm
    return bsm


def _blocks_at(bsm, M, rows, cols):
    """Blocks (rows[n], cols[n]) of a GPU matrix, from its pattern's CSR on the host."""
    rp, cc = M.pattern.to_host()
    out = []
    for i, j in zip(rows, cols):
        lo, hi = int(rp[i]), int(rp[i + 1])
        s = lo + int(np.searchsorted(cc[lo:hi], j))
        assert s < hi and cc[s] == j, (i, j)
        out.append(s)
    return M.blocks[torch.tensor(out, device=M.blocks.device)].cpu().numpy()


def _row_norms(M):
    rp, _ = M.pattern.to_host()
    sq = (M.blocks * M.blocks).sum(dim=(1, 2)).cpu().numpy()
    return np.sqrt(np.add.reduceat(sq, rp[:-1].astype(np.int64)))


@pytest.mark.parametrize("case", ["si512_b9_disp", "si4096_b9"])
def test_solve_matches_stored_oracle(bsm, case):
    g = golden(case)
    s = system(case)
    assert s.natoms == g["generator"]["natoms"] and s.b == g["generator"]["b"]
    cut = s.cutoffs
    say(f"[{case}] {s.natoms} atoms, b={s.b}: patterns and S, H")
    ctx = bsm.Context(0)
    pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
    PS = bsm.Pattern(ctx, pos, s.box, cut["S"], s.b)
    PZ = bsm.Pattern(ctx, pos, s.box, cut["Z"], s.b)
    PL = bsm.Pattern(ctx, pos, s.box, cut["L"], s.b)
    S, H, Z, L = bsm.Matrix(PS), bsm.Matrix(PS), bsm.Matrix(PZ), bsm.Matrix(PL)
    bsm.fill_blocks(S, s.S.rows, s.S.cols, s.S.blocks)
    bsm.fill_blocks(H, s.H.rows, s.H.cols, s.H.blocks)

    say(f"[{case}] Hotelling")
    gh = g["hotelling"]
    hr = bsm.hotelling_inverse(S, Z, max_iter=gh["max_iter"], tol=gh["tol"])
    assert hr.status == gh["status"] and hr.iterations == gh["iterations"]
    assert hr.alpha == pytest.approx(gh["alpha"], rel=1e-14)
    np.testing.assert_allclose(hr.residuals, gh["residuals"], rtol=1e-10)
    zs = g["Z_samples"]
    zg = _blocks_at(bsm, Z, zs["rows"], zs["cols"])
    zo = np.array(zs["blocks"]).reshape(zg.shape)
    zscale = max(g["Z_row_norms"])
    assert np.abs(zg - zo).max() <= 1e-10 * np.abs(zo).max()
    np.testing.assert_allclose(_row_norms(Z), g["Z_row_norms"], rtol=0, atol=1e-10 * zscale)

    say(f"[{case}] LNV")
    gl = g["lnv"]
    lnv = bsm.LNV(S, H, Z, L, s.n_electrons, tol_E=gl["tol_E"], init_from_z=True)
    ref = gl["iterations"]
    res = None
    for it in range(gl["max_iter"]):
        res = lnv.step()
        assert res.status == 0, (it, res.status)
        if it < len(ref):
            o = ref[it]
            assert abs(res.E - o["E"]) <= 1e-10 * abs(o["E"]), (it, res.E, o["E"])
            assert abs(res.N - o["N"]) <= 1e-10 * abs(o["N"]), (it, res.N, o["N"])
            if it < 6:
                assert abs(res.alpha - o["alpha"]) <= 1e-6 * abs(o["alpha"]), (it, res.alpha, o["alpha"])
                assert abs(res.mu - o["mu"]) <= 1e-8 * max(abs(o["mu"]), 1e-3), (it, res.mu, o["mu"])
        if res.converged:
            break
        if it >= len(ref):
            break
    say(f"[{case}] {it + 1} LNV iterations (oracle {len(ref)}), E = {res.E:.12f} (oracle {gl['E_final']:.12f})")
    assert res.converged and it + 1 == len(ref)
    assert abs(res.E - gl["E_final"]) <= 1e-10 * abs(gl["E_final"])
    ls = g["L_samples"]
    lg = _blocks_at(bsm, L, ls["rows"], ls["cols"])
    lo = np.array(ls["blocks"]).reshape(lg.shape)
    assert np.linalg.norm(lg - lo) <= 1e-8 * np.linalg.norm(lo)
    np.testing.assert_allclose(_row_norms(L), g["L_row_norms"], rtol=1e-8)
    if "idempotency_error" in gl:
        e = lnv.idempotency_error()
        say(f"[{case}] idempotency error {e:.6e} (oracle {gl['idempotency_error']:.6e})")
        assert abs(e - gl["idempotency_error"]) <= 1e-8 * gl["idempotency_error"]


def test_paired_launches_leave_the_solve_unchanged(bsm):
    """The solve with paired launches (default kernel) and without them (variant 3: the same ring
    tiles, single launches only) gives the same bits: Hotelling residuals, every LNV E, N and alpha,
    and the final L (512 displaced atoms, truncated L, S^-1 and S patterns, 8 LNV steps)."""
    s = system("si512_b9_disp")
    cut = s.cutoffs
    out = []
    for variant in (-1, 3):
        ctx = bsm.Context(0)
        ctx.set_product_variant(variant)
        say(f"paired launches: variant {variant}")
        pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
        PS = bsm.Pattern(ctx, pos, s.box, cut["S"], s.b)
        PZ = bsm.Pattern(ctx, pos, s.box, cut["Z"], s.b)
        PL = bsm.Pattern(ctx, pos, s.box, cut["L"], s.b)
        S, H, Z, L = bsm.Matrix(PS), bsm.Matrix(PS), bsm.Matrix(PZ), bsm.Matrix(PL)
        bsm.fill_blocks(S, s.S.rows, s.S.cols, s.S.blocks)
        bsm.fill_blocks(H, s.H.rows, s.H.cols, s.H.blocks)
        ctx.set_profiling(True)
        hr = bsm.hotelling_inverse(S, Z, max_iter=100, tol=1e-12)
        lnv = bsm.LNV(S, H, Z, L, s.n_electrons, init_from_z=True)
        steps = [lnv.step() for _ in range(8)]
        out.append((list(hr.residuals), [(r.E, r.N, r.alpha) for r in steps], L.blocks.cpu().numpy()))
        paired = sum(st["launches"] for st in ctx.product_stats() if st["products"] == 2)
        say(f"   paired launches: {paired}")
        assert (paired > 0) == (variant == -1)
        ctx.close()
    assert out[0][0] == out[1][0]
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2])
