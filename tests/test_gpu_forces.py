"""GPU forces (lnv_forces) against the oracle's on the same L and Z, and against
central differences of the GPU's own converged energies (geometry-smooth frames)."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu
KW = dict(displacement_sigma=0.05, smooth=True)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bsm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_08941_amd as bsm
    return bsm


def tens(x, ctx):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=ctx.device)


class GpuFrame:
    """Patterns, S, H and the derivative blocks of a frame on the GPU."""

    def __init__(self, bsm, ctx, s, derivatives=True):
        pos = tens(s.positions, ctx)
        self.P6 = bsm.Pattern(ctx, pos, s.box, s.cutoffs["S"], s.b)
        self.PZ = bsm.Pattern(ctx, pos, s.box, s.cutoffs["Z"], s.b)
        self.PL = bsm.Pattern(ctx, pos, s.box, s.cutoffs["L"], s.b)
        self.S, self.H = bsm.Matrix(self.P6), bsm.Matrix(self.P6)
        bsm.fill_blocks(self.S, s.S.rows, s.S.cols, s.S.blocks)
        bsm.fill_blocks(self.H, s.H.rows, s.H.cols, s.H.blocks)
        self.Z, self.L = bsm.Matrix(self.PZ), bsm.Matrix(self.PL)
        self.dS, self.dH = [], []
        if derivatives:
            for d in s.dS:
                m = bsm.Matrix(self.P6)
                bsm.fill_blocks(m, d.rows, d.cols, d.blocks)
                self.dS.append(m)
            for d in s.dH:
                m = bsm.Matrix(self.P6)
                bsm.fill_blocks(m, d.rows, d.cols, d.blocks)
                self.dH.append(m)

    def solve(self, bsm, s, tol_E):
        bsm.hotelling_inverse(self.S, self.Z, max_iter=100, tol=1e-12)
        lnv = bsm.LNV(self.S, self.H, self.Z, self.L, s.n_electrons, tol_E=tol_E)
        r = lnv.solve([(bsm.F64, 1000, tol_E, False)])
        assert r["converged"] and r["status"] == 0
        return lnv, r["E"]


@pytest.mark.parametrize("cells,b,cutoffs,steps", [(2, 4, synth.SMALL_CUTOFFS, 12), (2, 9, synth.SMALL_CUTOFFS, 12),
                                                   ((3, 3, 3), 4, synth.SMALL_CUTOFFS, 12),
                                                   ((4, 4, 4), 4, synth.BIG_CUTOFFS, 3)])
def test_forces_parity_same_L(bsm, cells, b, cutoffs, steps):
    # the oracle's L (after `steps` LNV steps) and Z loaded into the GPU state: forces within
    # 1e-10 of the largest component (only summation orders differ); 512 atoms on the 6/8/10 A
    # cutoffs: L, S^-1 and the overlap are truncated (191, 99 and 47 of 512 columns)
    s = synth.make_system("f", cells, b, cutoffs, 11, derivatives=True, **KW)
    say(f"forces parity {s.natoms} atoms b={b}")
    P6 = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    oS = O.from_blocks(P6, b, s.S.rows, s.S.cols, s.S.blocks)
    oH = O.from_blocks(P6, b, s.H.rows, s.H.cols, s.H.blocks)
    oZ = O.hotelling_inverse(oS, O.create_pattern(s.positions, s.box, s.cutoffs["Z"]), max_iter=100).Z
    st = O.lnv_init(oS, oH, oZ, O.create_pattern(s.positions, s.box, s.cutoffs["L"]), s.n_electrons, tol_E=1e-11)
    O.lnv_solve(st, [(O.F64, steps, 0.0, False)])   # any L: both sides differentiate at the same point
    Fo = O.lnv_forces(st, [O.from_blocks(P6, b, d.rows, d.cols, d.blocks) for d in s.dS],
                      [O.from_blocks(P6, b, d.rows, d.cols, d.blocks) for d in s.dH])
    ctx = bsm.Context(0)
    g = GpuFrame(bsm, ctx, s)
    g.Z.blocks.copy_(tens(oZ.blocks, ctx))
    g.L.blocks.copy_(tens(st.L.blocks, ctx))
    lnv = bsm.LNV(g.S, g.H, g.Z, g.L, s.n_electrons, init_from_z=False)
    F, mu = lnv.forces(g.dS, g.dH)
    say(f"   max |F| {np.abs(Fo).max():.3e}, max diff {np.abs(F - Fo).max():.3e}, mu {mu:.6f}")
    assert np.abs(F - Fo).max() < 1e-10 * np.abs(Fo).max()
    ctx.close()


def _safe_atom(s, radii, h):
    # an atom none of whose pair distances lies within 2h of a truncation radius, so that
    # moving it by h changes no pattern
    i, j, sh, d = synth.image_pairs(s.positions, s.box, max(radii) + 1.0)
    for a in range(s.natoms):
        da = d[i == a]
        if all(np.abs(da - r).min() > 2 * h for r in radii):
            return a
    raise AssertionError("no atom clear of the cutoffs")


@pytest.mark.parametrize("cells,cutoffs", [((4, 4, 4), synth.SMALL_CUTOFFS), (8, synth.BIG_CUTOFFS)])
def test_forces_match_gpu_energy_differences(bsm, cells, cutoffs):
    # at 512 and 4096 atoms (b = 9): one force component against central differences of
    # the GPU's converged energies, and translation invariance of all of them
    b, h, tol = 9, 1e-3, 1e-10
    s = synth.make_system("f", cells, b, cutoffs, 11, derivatives=True, **KW)
    say(f"forces vs energy differences {s.natoms} atoms")
    ctx = bsm.Context(0)
    g = GpuFrame(bsm, ctx, s)
    lnv, E0 = g.solve(bsm, s, tol)
    F, _ = lnv.forces(g.dS, g.dH)
    assert np.abs(F.sum(axis=0)).max() < 1e-9 * np.abs(F).max()
    atom = _safe_atom(s, (cutoffs["S"], cutoffs["L"]), h)
    c = int(np.argmax(np.abs(F[atom])))
    E = []
    for sign in (1.0, -1.0):
        e = np.zeros((s.natoms, 3))
        e[atom, c] = sign * h
        sd = synth.make_system("f", cells, b, cutoffs, 11, extra_displacement=e, **KW)
        gd = GpuFrame(bsm, ctx, sd, derivatives=False)
        E.append(gd.solve(bsm, sd, tol)[1])
        del gd
    fd = -(E[0] - E[1]) / (2 * h)
    say(f"   atom {atom} dir {c}: F {F[atom, c]:.9f}, -dE/dR {fd:.9f}")
    assert F[atom, c] == pytest.approx(fd, rel=2e-3, abs=1e-6)
    ctx.close()
