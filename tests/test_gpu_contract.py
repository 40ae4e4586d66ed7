"""GPU contraction to support functions (bsm_contract) against the oracle, and an LNV
solve of a contracted system against the oracle's."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bsm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_08941_amd as bsm
    return bsm


def onsite_coef(s, bc):
    # the bc lowest eigenvectors of every on-site H block (input preparation)
    on = s.H.rows == s.H.cols
    order = np.argsort(s.H.rows[on])
    return np.stack([np.linalg.eigh(blk)[1][:, :bc] for blk in s.H.blocks[on][order]])


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("cells,kind", [(2, "eig"), ((4, 4, 4), "eig"), ((3, 3, 3), "random")])
def test_contract_parity(bsm, cells, kind):
    s = synth.make_system("c", cells, 9, synth.SMALL_CUTOFFS, 5)
    say(f"contract {s.natoms} atoms ({kind} coefficients)")
    coef = onsite_coef(s, 4) if kind == "eig" else np.random.default_rng(3).normal(size=(s.natoms, 9, 4))
    ctx = bsm.Context(0)
    pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
    P9 = bsm.Pattern(ctx, pos, s.box, s.cutoffs["S"], 9)
    P4 = bsm.Pattern(ctx, pos, s.box, s.cutoffs["S"], 4)
    oP = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    for name in ("S", "H"):
        bl = getattr(s, name)
        M, Mc = bsm.Matrix(P9), bsm.Matrix(P4)
        bsm.fill_blocks(M, bl.rows, bl.cols, bl.blocks)
        bsm.contract(M, torch.tensor(coef, dtype=torch.float64, device=ctx.device).contiguous(), Mc)
        torch.cuda.synchronize()
        want = O.contract(O.from_blocks(oP, 9, bl.rows, bl.cols, bl.blocks), coef)
        assert rel_err(Mc.blocks.cpu().numpy(), want.blocks) < 1e-14
    with pytest.raises(bsm.BSMError):
        bsm.contract(bsm.Matrix(P4), torch.zeros((s.natoms, 4, 9), dtype=torch.float64, device=ctx.device),
                     bsm.Matrix(P9))   # more support functions than orbitals
    ctx.close()


@pytest.mark.parametrize("cells,cutoffs,steps", [(2, synth.SMALL_CUTOFFS, 10), ((4, 4, 4), synth.BIG_CUTOFFS, 4)])
def test_contracted_lnv_parity(bsm, cells, cutoffs, steps):
    # 9 orbitals contracted to 4 on-site support functions; Hotelling (10 steps) and LNV steps
    # of the contracted system on both sides: 64 atoms, and 512 atoms on the 6/8/10 A cutoffs
    # (L, S^-1 and the overlap truncated)
    s = synth.make_system("c", cells, 9, cutoffs, 5)
    coef = onsite_coef(s, 4)
    ctx = bsm.Context(0)
    pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
    P9 = bsm.Pattern(ctx, pos, s.box, s.cutoffs["S"], 9)
    P4 = bsm.Pattern(ctx, pos, s.box, s.cutoffs["S"], 4)
    ct = torch.tensor(coef, dtype=torch.float64, device=ctx.device).contiguous()
    Sc, Hc = bsm.Matrix(P4), bsm.Matrix(P4)
    for bl, out in ((s.S, Sc), (s.H, Hc)):
        M = bsm.Matrix(P9)
        bsm.fill_blocks(M, bl.rows, bl.cols, bl.blocks)
        bsm.contract(M, ct, out)
    Z = bsm.Matrix(bsm.Pattern(ctx, pos, s.box, s.cutoffs["Z"], 4))
    L = bsm.Matrix(bsm.Pattern(ctx, pos, s.box, s.cutoffs["L"], 4))
    bsm.hotelling_inverse(Sc, Z, max_iter=10, tol=0.0)
    lnv = bsm.LNV(Sc, Hc, Z, L, s.n_electrons)
    g = [lnv.step().E for _ in range(steps)]
    oP = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    oS = O.contract(O.from_blocks(oP, 9, s.S.rows, s.S.cols, s.S.blocks), coef)
    oH = O.contract(O.from_blocks(oP, 9, s.H.rows, s.H.cols, s.H.blocks), coef)
    oZ = O.hotelling_inverse(oS, O.create_pattern(s.positions, s.box, s.cutoffs["Z"]), max_iter=10, tol=0.0).Z
    st = O.lnv_init(oS, oH, oZ, O.create_pattern(s.positions, s.box, s.cutoffs["L"]), s.n_electrons)
    o = [O.lnv_step(st).E for _ in range(steps)]
    say(f"contracted LNV: E {g[-1]:.10f} (oracle {o[-1]:.10f})")
    np.testing.assert_allclose(g, o, rtol=1e-10)
    ctx.close()
