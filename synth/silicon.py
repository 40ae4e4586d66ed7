"""Seeded synthetic Si-like inputs for the block-sparse linear-scaling solver.

This module only *generates inputs*: atom positions, and the overlap S and
Hamiltonian H as lists of atom blocks.  It contains none of the solver's
arithmetic (no patterns, products, traces, inversion or minimisation), so
both the FP64 oracle and the HIP library can consume its output.

The paper's real workloads (bulk Si at up to 10^6 atoms, Background section
and Fig. 2c) use PAO bases and pseudopotentials that are not available here;
these arrays stand in for them with the same shape: diamond Si, one b x b
block per atom pair within the H/S range, 4 or 9 orbitals per atom.

Conventions
-----------
* Atoms are ordered cell by cell (cells in Morton order), basis atom last.
  Spatial neighbours are therefore near each other in the numbering.
* Blocks are Gamma-point folded: the block of atom pair (i, j) is the sum
  over every periodic image of j within range.
* Random numbers come from a counter-based hash (SplitMix64 finaliser) keyed
  by (seed, stream, pair, image, element), so a block does not depend on the
  order in which pairs are enumerated.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np

A_SI = 5.43  # conventional cubic lattice constant of Si, Angstrom
DIAMOND_BASIS = np.array(
    [[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
     [.25, .25, .25], [.25, .75, .75], [.75, .25, .75], [.75, .75, .25]], float)
# sp3 directions of sublattice A (basis 0-3); sublattice B uses the negatives.
TETRA = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) / np.sqrt(3.0)

T_BOND = 0.25      # Ha, hybrid-hybrid bond coupling
E_D = 0.5          # Ha, on-site energy of the d-like orbitals 4..8 (b = 9)
S_DECAY = 1.5      # Angstrom, decay length of off-site overlap and random H
S_AMP = 0.3        # overlap elements drawn uniformly in [-S_AMP, S_AMP]
STREAM_S, STREAM_H, STREAM_DISP = 0, 1, 2

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _mix(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = x + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        x = x ^ (x >> np.uint64(31))
    return x


def counter_uniform(*keys) -> np.ndarray:
    """Uniform [0, 1) doubles from a hash of integer key arrays (broadcast)."""
    keys = np.broadcast_arrays(*[np.asarray(k).astype(np.int64).astype(np.uint64) for k in keys])
    h = np.zeros(keys[0].shape, np.uint64)
    for k in keys:
        h = _mix(h ^ _mix(k))
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _morton3(q: np.ndarray, bits: int = 10) -> np.ndarray:
    code = np.zeros(len(q), np.int64)
    for bit in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> bit) & 1) << (3 * bit + d)
    return code


@dataclasses.dataclass
class BlockList:
    """A symmetric matrix as a list of atom blocks: block[n] sits at (rows[n], cols[n])."""
    rows: np.ndarray     # int32 (nnz,)
    cols: np.ndarray     # int32 (nnz,)
    blocks: np.ndarray   # float64 (nnz, b, b), row-major inside a block

    def to_dense(self, natoms: int) -> np.ndarray:
        b = self.blocks.shape[1]
        M = np.zeros((natoms * b, natoms * b))
        for r, c, blk in zip(self.rows, self.cols, self.blocks):
            M[r * b:(r + 1) * b, c * b:(c + 1) * b] += blk
        return M


@dataclasses.dataclass
class SiliconSystem:
    name: str
    positions: np.ndarray        # (N, 3) float64, Angstrom, inside [0, box)
    box: np.ndarray              # (3,) orthorhombic periodic box, Angstrom
    b: int                       # orbitals per atom (4 or 9)
    S: BlockList
    H: BlockList
    n_electrons: float           # 4 valence electrons per Si atom
    cutoffs: Dict[str, float]    # {"S","H","L","Z"} in Angstrom
    seed: int
    # derivatives (smooth systems, derivatives=True): dS[c] and dH[c] hold, block by block
    # on the S and H block lists, d S_ij / d R_j^c (= -d S_ij / d R_i^c for i != j; 0 for i == j)
    dS: Optional[List[BlockList]] = None
    dH: Optional[List[BlockList]] = None

    @property
    def natoms(self) -> int:
        return len(self.positions)


def diamond_positions(ncell: Tuple[int, int, int], a: float = A_SI):
    """Diamond lattice, ncell conventional cells per axis, Morton cell order."""
    n1, n2, n3 = ncell
    cells = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3),
                                 indexing="ij"), -1).reshape(-1, 3)
    cells = cells[np.argsort(_morton3(cells), kind="stable")]
    pos = ((cells[:, None, :] + DIAMOND_BASIS[None]) * a).reshape(-1, 3)
    sub = np.tile(np.array([0, 0, 0, 0, 1, 1, 1, 1]), len(cells))
    box = np.array([n1, n2, n3], float) * a
    return pos, box, sub


def image_pairs(pos: np.ndarray, box: np.ndarray, rcut: float):
    """All (i, j, image shift) with |r_j + shift*box - r_i| < rcut, excluding i == j at shift 0.

    Returns i, j (int64), shift (int64, (M,3)), d (float64).  Each unordered pair
    appears in both orders, with opposite shifts.
    """
    n = len(pos)
    if np.all(box > 2.0 * rcut + 1e-6) and n > 256:
        from scipy.spatial import cKDTree
        wrapped = np.mod(pos, box)
        tree = cKDTree(wrapped, boxsize=box)
        pr = tree.query_pairs(rcut, output_type="ndarray")
        i, j = pr[:, 0].astype(np.int64), pr[:, 1].astype(np.int64)
        dv = pos[j] - pos[i]
        shift = -np.rint(dv / box).astype(np.int64)
        dvec = dv + shift * box
        d = np.sqrt((dvec ** 2).sum(1))
        keep = d < rcut
        i, j, shift, d = i[keep], j[keep], shift[keep], d[keep]
        return (np.concatenate([i, j]), np.concatenate([j, i]),
                np.concatenate([shift, -shift]), np.concatenate([d, d]))
    m = np.ceil(rcut / box).astype(int)
    out_i, out_j, out_s, out_d = [], [], [], []
    for sx in range(-m[0], m[0] + 1):
        for sy in range(-m[1], m[1] + 1):
            for sz in range(-m[2], m[2] + 1):
                s = np.array([sx, sy, sz])
                dv = pos[None, :, :] + s * box - pos[:, None, :]
                d = np.sqrt((dv ** 2).sum(-1))
                ok = d < rcut
                if sx == 0 and sy == 0 and sz == 0:
                    np.fill_diagonal(ok, False)
                ii, jj = np.nonzero(ok)
                out_i.append(ii); out_j.append(jj)
                out_s.append(np.tile(s, (len(ii), 1))); out_d.append(d[ii, jj])
    return (np.concatenate(out_i).astype(np.int64), np.concatenate(out_j).astype(np.int64),
            np.concatenate(out_s).astype(np.int64), np.concatenate(out_d))


def _canonical(i, j, shift):
    """Key of an unordered image pair and whether (i, j, shift) is its transposed member."""
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    s = np.where((i <= j)[:, None], shift, -shift)
    # for i == j, pick between shift and -shift by the sign of the first non-zero component
    first = np.where(s[:, 0] != 0, s[:, 0], np.where(s[:, 1] != 0, s[:, 1], s[:, 2]))
    flip_self = (i == j) & (first < 0)
    s = np.where(flip_self[:, None], -s, s)
    transposed = (i > j) | flip_self
    return lo, hi, s, transposed


def _pair_random_blocks(seed, stream, i, j, shift, b, lo_val, hi_val):
    """b x b uniform blocks keyed by the unordered image pair; transposed for the mirror member."""
    lo, hi, s, transposed = _canonical(i, j, shift)
    e = np.arange(b * b)
    u = counter_uniform(seed, stream, lo[:, None], hi[:, None], s[:, 0:1] + 1000,
                        s[:, 1:2] + 1000, s[:, 2:3] + 1000, e[None, :])
    U = (lo_val + (hi_val - lo_val) * u).reshape(-1, b, b)
    U[transposed] = np.transpose(U[transposed], (0, 2, 1))
    return U


def _fold(i, j, blocks, natoms):
    """Sum image contributions into one block per (i, j); rows sorted, columns sorted."""
    key = i * natoms + j
    order = np.argsort(key, kind="stable")
    key, blocks = key[order], blocks[order]
    uk, start, count = np.unique(key, return_index=True, return_counts=True)
    # images of one pair added in list order, first + second + ... (most pairs have one)
    summed = blocks[start]
    for m in range(1, int(count.max()) if len(count) else 0):
        sel = np.nonzero(count > m)[0]
        summed[sel] += blocks[start[sel] + m]
    return (uk // natoms).astype(np.int32), (uk % natoms).astype(np.int32), summed


def _smooth_coefficients(seed, stream, b):
    """Seeded coefficient tensors of an orbital-pair function of the bond direction.

    U(r)_ab = [C0_ab + C1_abc r_c + C2_abcd r_c r_d] / 4 with C0 symmetric, C1
    antisymmetric and C2 symmetric in (a, b), so that U(-r) = U(r)^T: the block
    of the mirrored pair is the transpose, as a symmetric matrix needs.
    """
    a = np.arange(b)
    R0 = 2.0 * counter_uniform(seed, stream, 9000, a[:, None], a[None, :]) - 1.0
    c = np.arange(3)
    R1 = 2.0 * counter_uniform(seed, stream, 9001, a[:, None, None], a[None, :, None], c[None, None, :]) - 1.0
    R2 = 2.0 * counter_uniform(seed, stream, 9002, a[:, None, None, None], a[None, :, None, None],
                               c[None, None, :, None], c[None, None, None, :]) - 1.0
    C0 = 0.5 * (R0 + R0.T)
    C1 = 0.5 * (R1 - R1.transpose(1, 0, 2))
    C2 = 0.5 * (R2 + R2.transpose(1, 0, 2, 3))
    C2 = 0.5 * (C2 + C2.transpose(0, 1, 3, 2))
    return C0, C1, C2


def _smooth_blocks(coef, rhat):
    C0, C1, C2 = coef
    U = C0[None] + np.einsum("abc,nc->nab", C1, rhat) + np.einsum("abcd,nc,nd->nab", C2, rhat, rhat)
    return 0.25 * U


def _pair_vectors(pos, box, i, j, sh, d):
    return (pos[j] + sh * box - pos[i]) / d[:, None]


def _smooth_pair_derivative(coef, pos, box, i, j, sh, d):
    """d/dr_c of exp(-d / S_DECAY) U(r_hat) at the pair vector r (= r_j + shift box - r_i),
    shape (n, 3, b, b): the radial factor's derivative times U plus the angular part,
    dU/dr_hat_e (delta_ec - r_hat_e r_hat_c) / d."""
    _, C1, C2 = coef
    rh = _pair_vectors(pos, box, i, j, sh, d)
    U = _smooth_blocks(coef, rh)
    dU = 0.25 * (C1[None] + 2.0 * np.einsum("abef,nf->nabe", C2, rh))
    proj = (np.eye(3)[None] - rh[:, :, None] * rh[:, None, :]) / d[:, None, None]
    g = np.einsum("nabe,nec->ncab", dU, proj) - (rh / S_DECAY)[:, :, None, None] * U[:, None]
    return np.exp(-d / S_DECAY)[:, None, None, None] * g


def make_system(name: str, ncell, b: int, cutoffs: Dict[str, float], seed: int,
                displacement_sigma: float = 0.0, s_amp: float = S_AMP,
                h_random: bool = True, smooth: bool = False,
                extra_displacement: Optional[np.ndarray] = None,
                derivatives: bool = False) -> SiliconSystem:
    """Diamond-Si system with seeded S and gapped tight-binding-like H.

    S: identity on site; off site exp(-d/1.5 A) * U, U uniform in [-0.3, 0.3],
       for every image within the S cutoff.
    H: V_bond + V_d + V_rand.  V_bond couples the two sp3-like hybrids (orbitals
       0..3) facing each other across every nearest-neighbour bond with -t; V_d puts
       orbitals 4..8 at +0.5 Ha; V_rand is exp(-d/1.5 A) * uniform[-1, 1] within the
       H cutoff, scaled so that its largest absolute row sum is t/2, which keeps
       a gap around zero energy with exactly 2 N occupied states.

    s_amp = 0 gives S = I; h_random = False drops V_rand (both only for tests
    with closed-form answers); a large s_amp makes S indefinite.

    smooth = True makes every block a function of the pair geometry alone, so
    that S, H (and hence the density matrix) vary smoothly with displacements
    and can be learned from geometry: the uniform off-site factors become
    seeded orbital-pair functions of the bond direction (_smooth_coefficients),
    the on-site part of V_rand is one seeded symmetric block shared by all
    atoms, and the V_rand scale is fixed on the undisplaced lattice.

    extra_displacement (N, 3) is added to the positions after the seeded
    displacements (finite differences); derivatives = True (smooth only) also
    returns the derivative blocks dS, dH of every S and H block with respect to
    its column atom's position.
    """
    ncell = (ncell,) * 3 if np.isscalar(ncell) else tuple(ncell)
    ideal, box, sub = diamond_positions(ncell)
    natoms = len(ideal)
    pos = ideal.copy()
    if displacement_sigma > 0:
        # Box-Muller from the counter generator, keyed by (seed, atom, component)
        idx = np.arange(natoms)[:, None]
        comp = np.arange(3)[None, :]
        u1 = counter_uniform(seed, STREAM_DISP, idx, comp, 0)
        u2 = counter_uniform(seed, STREAM_DISP, idx, comp, 1)
        gauss = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2 * np.pi * u2)
        pos = pos + displacement_sigma * gauss
    if extra_displacement is not None:
        pos = pos + np.asarray(extra_displacement, float)
    pos = np.mod(pos, box)
    if derivatives and not smooth:
        raise ValueError("derivative blocks need the geometry-smooth generator (smooth=True)")

    rS, rH = cutoffs["S"], cutoffs["H"]
    rmax = max(rS, rH)
    i, j, sh, d = image_pairs(pos, box, rmax)

    # ---- S -------------------------------------------------------------
    inS = d < rS
    if smooth:
        offS = (s_amp * np.exp(-d[inS] / S_DECAY))[:, None, None] * _smooth_blocks(
            _smooth_coefficients(seed, STREAM_S, b), _pair_vectors(pos, box, i[inS], j[inS], sh[inS], d[inS]))
    else:
        offS = np.exp(-d[inS] / S_DECAY)[:, None, None] * _pair_random_blocks(
            seed, STREAM_S, i[inS], j[inS], sh[inS], b, -s_amp, s_amp)
    diag = np.arange(natoms)
    eye = np.broadcast_to(np.eye(b), (natoms, b, b))
    S = BlockList(*_fold(np.concatenate([diag, i[inS]]), np.concatenate([diag, j[inS]]),
                         np.concatenate([eye, offS]), natoms))

    # ---- H -------------------------------------------------------------
    inH = d < rH
    if smooth:
        coefH = _smooth_coefficients(seed, STREAM_H, b)

        def vrand(p, ii, jj, ss, dd):
            off = np.exp(-dd / S_DECAY)[:, None, None] * _smooth_blocks(coefH, _pair_vectors(p, box, ii, jj, ss, dd))
            on = np.broadcast_to(coefH[0], (natoms, b, b))
            return _fold(np.concatenate([diag, ii]), np.concatenate([diag, jj]), np.concatenate([on, off]), natoms)

        ri, rj, Vr = vrand(pos, i[inH], j[inH], sh[inH], d[inH])
        scale_pairs = image_pairs(ideal, box, rH)
        Ri, Rj, Vi = vrand(ideal, *scale_pairs)
    else:
        Vr_off = np.exp(-d[inH] / S_DECAY)[:, None, None] * _pair_random_blocks(
            seed, STREAM_H, i[inH], j[inH], sh[inH], b, -1.0, 1.0)
        e = np.arange(b * b)
        u_on = counter_uniform(seed, STREAM_H, diag[:, None], diag[:, None], 1000, 1000, 1000,
                               e[None, :]).reshape(natoms, b, b)
        Von = -1.0 + 2.0 * u_on
        Von = 0.5 * (Von + np.transpose(Von, (0, 2, 1)))
        ri, rj, Vr = _fold(np.concatenate([diag, i[inH]]), np.concatenate([diag, j[inH]]),
                           np.concatenate([Von, Vr_off]), natoms)
        Ri, Vi = ri, Vr
    rowsum = np.zeros(natoms * b)
    np.add.at(rowsum, (Ri[:, None] * b + np.arange(b)[None, :]).ravel(),
              np.abs(Vi).sum(axis=2).ravel())
    Vr = Vr * ((0.5 * T_BOND) / rowsum.max() if h_random else 0.0)

    # bonds: topological nearest neighbours of the ideal lattice
    bi, bj, bsh, bd = image_pairs(ideal, box, 0.5 * (2.3513 + 3.8396))
    vec = ideal[bj] + bsh * box - ideal[bi]
    vec /= np.linalg.norm(vec, axis=1)[:, None]
    sign = np.where(sub[bi] == 0, 1.0, -1.0)
    hyb = np.argmax((sign[:, None] * vec) @ TETRA.T, axis=1)
    Vb = np.zeros((len(bi), b, b))
    Vb[np.arange(len(bi)), hyb, hyb] = -T_BOND
    Vd = np.zeros((natoms, b, b))
    if b == 9:
        Vd[:, np.arange(4, 9), np.arange(4, 9)] = E_D
    H = BlockList(*_fold(np.concatenate([ri, bi.astype(np.int32), diag]),
                         np.concatenate([rj, bj.astype(np.int32), diag]),
                         np.concatenate([Vr, Vb, Vd]), natoms))
    dS = dH = None
    if derivatives:
        # the same folds as S and H with derivative blocks in place of the blocks (zero for the
        # geometry-independent parts and for images of an atom with itself)
        zero = np.zeros((natoms, b, b))
        gS = s_amp * _smooth_pair_derivative(_smooth_coefficients(seed, STREAM_S, b), pos, box,
                                             i[inS], j[inS], sh[inS], d[inS])
        gS[i[inS] == j[inS]] = 0.0
        gH = _smooth_pair_derivative(coefH, pos, box, i[inH], j[inH], sh[inH], d[inH])
        gH[i[inH] == j[inH]] = 0.0
        scale = (0.5 * T_BOND) / rowsum.max() if h_random else 0.0
        dS, dH = [], []
        for c in range(3):
            dS.append(BlockList(*_fold(np.concatenate([diag, i[inS]]), np.concatenate([diag, j[inS]]),
                                       np.concatenate([zero, gS[:, c]]), natoms)))
            hr, hc, hv = _fold(np.concatenate([diag, i[inH]]), np.concatenate([diag, j[inH]]),
                               np.concatenate([zero, scale * gH[:, c]]), natoms)
            dH.append(BlockList(*_fold(np.concatenate([hr, bi.astype(np.int32), diag]),
                                       np.concatenate([hc, bj.astype(np.int32), diag]),
                                       np.concatenate([hv, np.zeros_like(Vb), zero]), natoms)))
    return SiliconSystem(name=name, positions=pos, box=box, b=b, S=S, H=H,
                         n_electrons=4.0 * natoms, cutoffs=dict(cutoffs), seed=seed, dS=dS, dH=dH)


# ---------------------------------------------------------------------------
# Workloads.  Cutoffs in Angstrom.  Sizes follow the Si runs the paper's
# weak-scaling figure is quoted on, scaled to one GPU.
# ---------------------------------------------------------------------------
SMALL_CUTOFFS = {"S": 6.0, "H": 6.0, "L": 8.0, "Z": 8.0}
BIG_CUTOFFS = {"S": 6.0, "H": 6.0, "L": 10.0, "Z": 8.0}


def si64_b4(seed: int = 2205) -> SiliconSystem:
    """64 atoms (2x2x2 cells, box 10.86 A), 4 orbitals per atom."""
    return make_system("si64_b4", 2, 4, SMALL_CUTOFFS, seed)


def si4096_b9(seed: int = 2205) -> SiliconSystem:
    """4096 atoms (8x8x8 cells, box 43.44 A), 9 orbitals per atom."""
    return make_system("si4096_b9", 8, 9, BIG_CUTOFFS, seed)


def displaced_frame(ncell, b: int, seed: int, sigma: float = 0.05, cutoffs=None) -> SiliconSystem:
    """A geometry-smooth frame: diamond Si with seeded Gaussian displacements of width sigma (A)."""
    ncell = (ncell,) * 3 if np.isscalar(ncell) else tuple(ncell)
    return make_system(f"si{8 * ncell[0] * ncell[1] * ncell[2]}_b{b}_frame{seed}", ncell, b,
                       dict(cutoffs or BIG_CUTOFFS), seed, displacement_sigma=sigma, smooth=True)


def random_blocks(nnz: int, b: int, seed: int, stream: int = 7, scale: float = 1.0) -> np.ndarray:
    """Seeded uniform[-scale, scale] blocks, for feeding kernels arbitrary operands."""
    u = counter_uniform(seed, stream, np.arange(nnz * b * b))
    return (scale * (2.0 * u - 1.0)).reshape(nnz, b, b)


def batch_cells(count: int = 64, seed: int = 2205, lo: int = 512, hi: int = 4096, min_cells: int = 4):
    """Cell counts and orbitals per atom of a batch of uneven systems.

    Target sizes uniform in [lo, hi] atoms, b = 4 or 9 by a seeded coin; each
    system is the orthorhombic n1 x n2 x n3 block of conventional cells (every
    n_i >= min_cells) whose 8 n1 n2 n3 atoms are closest to its target.
    """
    shapes = [(a, b, c) for a in range(min_cells, 17) for b in range(a, 17) for c in range(b, 17)]
    out = []
    for k in range(count):
        target = lo + (hi - lo) * float(counter_uniform(seed, 11, k))
        orb = 9 if counter_uniform(seed, 12, k) >= 0.5 else 4
        best = min(shapes, key=lambda s: (abs(8 * s[0] * s[1] * s[2] - target), s))
        out.append((best, orb))
    return out
