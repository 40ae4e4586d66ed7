"""FP64 CPU oracle for the block-sparse LNV / Hotelling hot path.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline may import this package; the HIP product path never does.  It shares
no code with the HIP library (`paper_2205_08941_amd`), and neither imports the
other.  Only `synth` (seeded inputs, no solver arithmetic) feeds both.

What it computes, and where it comes from:

* block-sparse storage and truncated products -- the paper's statement that
  the solver rests on sparse matrix storage and operations exploiting locality
  (Background and Current Status); the operations are defined in `oracle.c`;
* Hotelling's iteration Z <- 2Z - Z S Z for the overlap inverse -- the paper's
  "linear scaling inversion of the overlap matrix" (Development Priorities),
  by the textbook iteration of Hotelling (1943) / Schulz (1933);
* the inverse square root S^-1/2 (and S^1/2) of the same overlap matrix by
  the coupled Newton-Schulz iteration (Higham 1997), the companion of that
  inversion for symmetric (Loewdin) orthogonalisation;
* forces -dOmega/dR at the converged density matrix (Hellmann-Feynman and
  energy-density-matrix terms), from derivative blocks of S and H;
* contraction of S and H to a few support functions per atom (the on-site
  equivalent of multi-site support functions, Development Priorities);
* LNV density-matrix minimisation, K = 3LSL - 2LSLSL -- the paper's linear
  scaling O(N) ground-state solver (Background; Meeting the Exascale
  Challenges), in the non-orthogonal form of Li, Nunes and Vanderbilt (1993)
  and Nunes and Vanderbilt (1994), with conjugate gradients, an exact cubic
  line search and a constant-electron-number projection.

Parity pins (tests/test_oracle_*.py): dense masked matmul, np.trace, the dense
inverse and the closed-form Hotelling residual, finite differences of the
LNV energy, the generalised eigenvalue sum for untruncated cutoffs, the
bond-projector closed form E = -4 N t, and the diamond shell counts.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "_liboracle.so")

# status codes (same meaning as the library's documented codes)
OK, EINVAL, ENOMEM, EPATTERN, EHIP, ENONFINITE, EDIVERGED, ENOTCONV, ERUNAWAY = \
    0, -1, -2, -3, -4, -5, -6, -7, -8


_HOST_TAG = _SO + ".host"


def _host_cpu() -> str:
    """The CPU model of this machine (the library is tuned for it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc -O3 -march=native, OpenMP and no FMA contraction.

    Without -ffast-math gcc neither reassociates nor contracts, so the results do
    not depend on the instruction set; -march=native only makes the timed CPU
    baseline representative.  The library is rebuilt on a machine with another
    CPU model (a tag file beside it records the model it was built for)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
        with open(_HOST_TAG, "w") as f:
            f.write(_host_cpu())
    return _SO


def _built_here() -> bool:
    try:
        return (os.path.getmtime(_SO) >= os.path.getmtime(_SRC)
                and open(_HOST_TAG).read() == _host_cpu())
    except OSError:
        return False


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not _built_here():
            build(force=True)
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.orc_pattern_count.restype = ctypes.c_int64
        L.orc_pattern_count.argtypes = [ctypes.c_int, P, P, ctypes.c_double, P]
        L.orc_pattern_fill.restype = None
        L.orc_pattern_fill.argtypes = [ctypes.c_int, P, P, ctypes.c_double, P, P]
        L.orc_multiply.restype = None
        L.orc_multiply.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P, P, P, P, P,
                                   ctypes.c_double, P, P, P, ctypes.c_int, ctypes.c_int]
        L.orc_count_triples.restype = None
        L.orc_count_triples.argtypes = [ctypes.c_int, P, P, P, P, P, P, P]
        L.orc_multiply_mixed.restype = None
        L.orc_multiply_mixed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P, P, P,
                                         P, P, ctypes.c_double, P, P, P, ctypes.c_int, ctypes.c_int]
        L.orc_round_bf16.restype = ctypes.c_float
        L.orc_round_bf16.argtypes = [ctypes.c_float]
        L.orc_trace_product.restype = ctypes.c_double
        L.orc_trace_product.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
        _lib_handle = L
    return _lib_handle


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Block-sparse storage
# ---------------------------------------------------------------------------
class Pattern:
    """P_r: atom pairs with minimum-image distance below `cutoff`, diagonal included.

    Block CSR: rowptr (int64, n+1), cols (int32, ascending per row).
    """

    def __init__(self, natoms, rowptr, cols, cutoff, positions, box):
        self.natoms = int(natoms)
        self.rowptr = np.ascontiguousarray(rowptr, np.int64)
        self.cols = np.ascontiguousarray(cols, np.int32)
        self.cutoff = float(cutoff)
        self.positions = np.ascontiguousarray(positions, np.float64)
        self.box = np.ascontiguousarray(box, np.float64)
        self._tmap = None

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def rows(self) -> np.ndarray:
        return np.repeat(np.arange(self.natoms, dtype=np.int32), np.diff(self.rowptr))

    def keys(self) -> np.ndarray:
        return self.rows().astype(np.int64) * self.natoms + self.cols

    def find(self, rows, cols) -> np.ndarray:
        """Slots of (rows, cols), -1 where absent."""
        keys = self.keys()
        q = np.asarray(rows, np.int64) * self.natoms + np.asarray(cols, np.int64)
        s = np.searchsorted(keys, q)
        s = np.minimum(s, len(keys) - 1)
        return np.where(keys[s] == q, s, -1)

    def transpose_map(self) -> np.ndarray:
        """Slot of (j, i) for every slot (i, j); the pattern is symmetric by construction."""
        if self._tmap is None:
            t = self.find(self.cols, self.rows())
            if np.any(t < 0):
                raise ValueError("pattern is not symmetric")
            self._tmap = t
        return self._tmap

    def diag_slots(self) -> np.ndarray:
        return self.find(np.arange(self.natoms), np.arange(self.natoms))


def create_pattern(positions, box, cutoff) -> Pattern:
    """Brute force over all atom pairs, strict d^2 < r^2 under the minimum-image rule."""
    pos = np.ascontiguousarray(positions, np.float64)
    bx = np.ascontiguousarray(box, np.float64)
    n = len(pos)
    cnt = np.zeros(n, np.int64)
    L = _lib()
    L.orc_pattern_count(n, _p(pos), _p(bx), float(cutoff), _p(cnt))
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(cnt, out=rowptr[1:])
    cols = np.zeros(int(rowptr[-1]), np.int32)
    L.orc_pattern_fill(n, _p(pos), _p(bx), float(cutoff), _p(rowptr), _p(cols))
    return Pattern(n, rowptr, cols, cutoff, pos, bx)


class Matrix:
    """Block-sparse matrix: pattern + blocks (nnz, b, b) in CSR order."""

    def __init__(self, pattern: Pattern, b: int, blocks: Optional[np.ndarray] = None):
        self.pattern = pattern
        self.b = int(b)
        if blocks is None:
            blocks = np.zeros((pattern.nnz, b, b))
        self.blocks = np.ascontiguousarray(blocks, np.float64)
        assert self.blocks.shape == (pattern.nnz, b, b)

    def copy(self) -> "Matrix":
        return Matrix(self.pattern, self.b, self.blocks.copy())

    def zeros_like(self) -> "Matrix":
        return Matrix(self.pattern, self.b)

    def to_dense(self) -> np.ndarray:
        n, b = self.pattern.natoms, self.b
        D = np.zeros((n, b, n, b))
        D[self.pattern.rows(), :, self.pattern.cols, :] = self.blocks
        return D.reshape(n * b, n * b)

    @property
    def nrows(self) -> int:
        return self.pattern.natoms * self.b


def from_blocks(pattern: Pattern, b: int, rows, cols, blocks) -> Matrix:
    """Place a list of blocks into a pattern; every block must fall inside it."""
    s = pattern.find(rows, cols)
    if np.any(s < 0):
        raise ValueError("block outside the pattern")
    M = Matrix(pattern, b)
    np.add.at(M.blocks, s, blocks)
    return M


def from_dense(pattern: Pattern, b: int, D: np.ndarray) -> Matrix:
    n = pattern.natoms
    D4 = D.reshape(n, b, n, b)
    return Matrix(pattern, b, D4[pattern.rows(), :, pattern.cols, :])


def identity(pattern: Pattern, b: int, alpha: float = 1.0) -> Matrix:
    M = Matrix(pattern, b)
    M.blocks[pattern.diag_slots()] = alpha * np.eye(b)
    return M


def mask_copy(src: Matrix, pattern: Pattern) -> Matrix:
    """mask_P(src): blocks of src kept where they fall in `pattern`, zero elsewhere."""
    out = Matrix(pattern, src.b)
    s = src.pattern.find(pattern.rows(), pattern.cols)
    ok = s >= 0
    out.blocks[ok] = src.blocks[s[ok]]
    return out


def multiply_truncate(alpha: float, A: Matrix, B: Matrix, beta: float, C: Matrix,
                      row_begin: int = 0, row_end: Optional[int] = None) -> None:
    """C <- alpha * mask_{P_C}(A B) + beta * C (in place), rows [row_begin, row_end)."""
    n = C.pattern.natoms
    if not (A.pattern.natoms == B.pattern.natoms == n and A.b == B.b == C.b):
        raise ValueError("pattern mismatch")
    if row_end is None:
        row_end = n
    _lib().orc_multiply(n, C.b, float(alpha),
                        _p(A.pattern.rowptr), _p(A.pattern.cols), _p(A.blocks),
                        _p(B.pattern.rowptr), _p(B.pattern.cols), _p(B.blocks),
                        float(beta), _p(C.pattern.rowptr), _p(C.pattern.cols), _p(C.blocks),
                        int(row_begin), int(row_end))


F64, F32, BF16 = 0, 1, 2


def multiply_truncate_mixed(prec: int, alpha: float, A: Matrix, B: Matrix, beta: float, C: Matrix,
                            row_begin: int = 0, row_end: Optional[int] = None) -> None:
    """C <- alpha mask(A B) + beta C with inputs rounded to FP32 (prec 1) or BF16 (prec 2),
    FP32 fused multiply-add accumulation in (k, m) order, FP64 output."""
    if prec == F64:
        return multiply_truncate(alpha, A, B, beta, C, row_begin, row_end)
    n = C.pattern.natoms
    if not (A.pattern.natoms == B.pattern.natoms == n and A.b == B.b == C.b):
        raise ValueError("pattern mismatch")
    if row_end is None:
        row_end = n
    _lib().orc_multiply_mixed(n, C.b, int(prec), float(alpha),
                              _p(A.pattern.rowptr), _p(A.pattern.cols), _p(A.blocks),
                              _p(B.pattern.rowptr), _p(B.pattern.cols), _p(B.blocks),
                              float(beta), _p(C.pattern.rowptr), _p(C.pattern.cols), _p(C.blocks),
                              int(row_begin), int(row_end))


def round_bf16(x: float) -> float:
    """FP32 -> BF16 -> FP32, round to nearest even (the oracle's rounding)."""
    return float(_lib().orc_round_bf16(float(x)))


def product(A: Matrix, B: Matrix, pattern: Pattern, prec: int = F64) -> Matrix:
    C = Matrix(pattern, A.b)
    multiply_truncate_mixed(prec, 1.0, A, B, 0.0, C)
    return C


def count_triples(PA: Pattern, PB: Pattern, PC: Pattern) -> np.ndarray:
    """Block triples (i,k,j) of mask_C(A B), per row of C (int64)."""
    out = np.zeros(PC.natoms, np.int64)
    _lib().orc_count_triples(PC.natoms, _p(PA.rowptr), _p(PA.cols), _p(PB.rowptr),
                             _p(PB.cols), _p(PC.rowptr), _p(PC.cols), _p(out))
    return out


def trace_product(A: Matrix, B: Matrix) -> float:
    """Tr(A B), FP64."""
    return float(_lib().orc_trace_product(A.pattern.natoms, A.b,
                                          _p(A.pattern.rowptr), _p(A.pattern.cols), _p(A.blocks),
                                          _p(B.pattern.rowptr), _p(B.pattern.cols), _p(B.blocks)))


def trace(A: Matrix) -> float:
    d = A.pattern.diag_slots()
    return float(np.trace(A.blocks[d], axis1=1, axis2=2).sum())


def dot(A: Matrix, B: Matrix) -> float:
    """Frobenius inner product <A, B> of two matrices on the same pattern."""
    assert A.pattern is B.pattern
    return float(np.dot(A.blocks.ravel(), B.blocks.ravel()))


def transpose(M: Matrix) -> Matrix:
    t = M.pattern.transpose_map()
    return Matrix(M.pattern, M.b, np.transpose(M.blocks[t], (0, 2, 1)))


def symmetrize(M: Matrix) -> Matrix:
    """(M + M^T) / 2, blockwise: (i,j) <- (M_ij + M_ji^T) / 2."""
    T = transpose(M)
    return Matrix(M.pattern, M.b, 0.5 * (M.blocks + T.blocks))


def derived_pattern(P: Pattern, cutoff: float) -> Pattern:
    return create_pattern(P.positions, P.box, cutoff)


# ---------------------------------------------------------------------------
# Hotelling / Schulz iteration for the overlap inverse
# ---------------------------------------------------------------------------
@dataclass
class HotellingResult:
    Z: Matrix
    status: int
    iterations: int
    residuals: List[float]
    alpha: float


def gershgorin_bound(S: Matrix) -> float:
    """max over scalar rows of sum_j |S_ij|: an upper bound of the spectrum of S."""
    n, b = S.pattern.natoms, S.b
    rowsum = np.zeros(n * b)
    rr = S.pattern.rows()
    np.add.at(rowsum, (rr[:, None] * b + np.arange(b)[None, :]).ravel(),
              np.abs(S.blocks).sum(axis=2).ravel())
    return float(rowsum.max())


def _hotelling_residual(T: Matrix, nb: int) -> float:
    """||I - Z S||_F from T = Z S, summed elementwise over (T - I)^2.

    (Equal to sqrt(N_b - 2 Tr T + ||T||_F^2), but that form cancels to about
    1e-13 N_b absolute in r^2, which hides residuals below ~1e-6.)
    """
    R = T.blocks.copy()
    R[T.pattern.diag_slots()] -= np.eye(T.b)
    r2 = float(np.dot(R.ravel(), R.ravel()))
    return math.sqrt(r2) if math.isfinite(r2) else float("nan")


HOTELLING_PROGRESS = 0.99   # an update must cut the residual by at least 1 %


def hotelling_inverse(S: Matrix, z_pattern: Pattern, max_iter: int = 100, tol: float = 1e-12,
                      Z0: Optional[Matrix] = None) -> HotellingResult:
    """Truncated Hotelling iteration Z <- sym(mask_Z(2Z - (Z S) Z)).

    Start Z0 = I / rho with rho the Gershgorin bound of S (so 0 < rho^-1 lambda <= 1).
    T = Z S is kept on P(r_Z + r_S), which holds it exactly, so the residual
    ||I - Z S||_F is exact (summed elementwise over T - I).
    Stops: residual < tol sqrt(N_b) (tol > 0); max_iter updates; no progress (the
    next residual is above 0.99 times the current one: keep the current Z,
    accepted when its residual is at most 0.1 sqrt(N_b), the truncation floor,
    else divergence).  Away from the floor an update at least squares the
    error, so only the floor or divergence stop it this way.
    """
    nb = S.nrows
    PT = derived_pattern(z_pattern, z_pattern.cutoff + S.pattern.cutoff)
    alpha = 1.0 / gershgorin_bound(S)
    Z = identity(z_pattern, S.b, alpha) if Z0 is None else mask_copy(Z0, z_pattern)
    T = product(Z, S, PT)
    r = _hotelling_residual(T, nb)
    if not math.isfinite(r):
        return HotellingResult(Z, ENONFINITE, 0, [r], alpha)
    hist, it, status = [r], 0, OK
    while True:
        if tol > 0 and r < tol * math.sqrt(nb):
            status = OK
            break
        if it == max_iter:
            status = ENOTCONV if tol > 0 else OK
            break
        M = product(T, Z, z_pattern)
        Znew = symmetrize(Matrix(z_pattern, S.b, 2.0 * Z.blocks - M.blocks))
        Tnew = product(Znew, S, PT)
        rnew = _hotelling_residual(Tnew, nb)
        if not math.isfinite(rnew):
            status = ENONFINITE
            break
        if rnew >= HOTELLING_PROGRESS * r:   # no real progress: the floor (accept) or divergence
            status = OK if r <= 0.1 * math.sqrt(nb) else EDIVERGED
            break
        Z, T, r = Znew, Tnew, rnew
        it += 1
        hist.append(r)
    return HotellingResult(Z, status, it, hist, alpha)


# ---------------------------------------------------------------------------
# Inverse square root of the overlap matrix (coupled Newton-Schulz)
# ---------------------------------------------------------------------------
@dataclass
class InvSqrtResult:
    Z: Matrix              # S^-1/2 on the Z pattern
    Y: Matrix              # S^1/2 on the same pattern
    status: int
    iterations: int
    residuals: List[float]
    alpha: float           # 1 / rho, rho the Gershgorin bound of S


def inverse_sqrt(S: Matrix, z_pattern: Pattern, max_iter: int = 100, tol: float = 1e-12) -> InvSqrtResult:
    """Truncated coupled Newton-Schulz iteration for S^-1/2 and S^1/2.

    The paper names linear-scaling inversion of the overlap matrix as key
    (Development Priorities); this is the inverse-square-root companion of the
    Hotelling iteration, in the coupled form analysed by Higham (1997,
    "Stable iterations for the matrix square root"): with A = S / rho (rho the
    Gershgorin bound, so the spectrum of A lies in (0, 1] for SPD S),
    Y0 = mask_Z(A), Z0 = I and, per update,
        P = Z Y,  T = (3 I - P) / 2,  Y <- Y T,  Z <- T Z,
    so that Y -> A^1/2 and Z -> A^-1/2.  Truncation as for Hotelling: only the
    iterates Y and Z are truncated (to the Z pattern, then symmetrised
    blockwise); P and T are held exactly on P(2 r_Z).  The residual
    ||I - Z Y||_F is summed elementwise over P - I.  The stop rules are
    Hotelling's (tolerance, max_iter, no real progress: accepted at or below
    0.1 sqrt(N_b), else divergence).  Returned: Z / sqrt(rho) = S^-1/2 and
    sqrt(rho) Y = S^1/2.
    """
    nb, b = S.nrows, S.b
    P2 = derived_pattern(z_pattern, 2.0 * z_pattern.cutoff)
    rho = gershgorin_bound(S)
    alpha = 1.0 / rho
    Y = mask_copy(S, z_pattern)
    Y = Matrix(z_pattern, b, alpha * Y.blocks)
    Z = identity(z_pattern, b)
    P = product(Z, Y, P2)
    r = _hotelling_residual(P, nb)
    hist, it, status = [r], 0, OK
    if not math.isfinite(r):
        status = ENONFINITE
    while status == OK:
        if tol > 0 and r < tol * math.sqrt(nb):
            break
        if it == max_iter:
            status = ENOTCONV if tol > 0 else OK
            break
        T = Matrix(P2, b, -0.5 * P.blocks)
        T.blocks[P2.diag_slots()] += 1.5 * np.eye(b)
        Ynew = symmetrize(product(Y, T, z_pattern))
        Znew = symmetrize(product(T, Z, z_pattern))
        Pnew = product(Znew, Ynew, P2)
        rnew = _hotelling_residual(Pnew, nb)
        if not math.isfinite(rnew):
            status = ENONFINITE
            break
        if rnew >= HOTELLING_PROGRESS * r:   # no real progress: the floor (accept) or divergence
            status = OK if r <= 0.1 * math.sqrt(nb) else EDIVERGED
            break
        Y, Z, P, r = Ynew, Znew, Pnew, rnew
        it += 1
        hist.append(r)
    zs, ys = 1.0 / math.sqrt(rho), math.sqrt(rho)
    return InvSqrtResult(Matrix(z_pattern, b, zs * Z.blocks), Matrix(z_pattern, b, ys * Y.blocks),
                         status, it, hist, alpha)


# ---------------------------------------------------------------------------
# LNV density-matrix minimisation
# ---------------------------------------------------------------------------
CANONICAL, GRAND = 0, 1


def lnv_initial_scale(nb: int, n_electrons: float, t2: float, t3: float) -> float:
    """c such that N(c Z) = 2 (3 c^2 t2 - 2 c^3 t3) = N_e, the root nearest c0.

    c0 solves 3 c^2 - 2 c^3 = N_e / (2 N_b) (the value for Z = S^-1 exactly).
    Both are found by Newton's method from the middle of the bracket [0, 1]
    where 3c^2 - 2c^3 is monotone.
    """
    nu = n_electrons / (2.0 * nb)

    def newton(f, df, x):
        for _ in range(100):
            step = f(x) / df(x)
            x -= step
            if abs(step) <= 1e-16 * max(1.0, abs(x)):
                break
        return x

    c0 = newton(lambda c: 3 * c * c - 2 * c ** 3 - nu, lambda c: 6 * c - 6 * c * c, 0.5)
    c = newton(lambda c: 2 * (3 * c * c * t2 - 2 * c ** 3 * t3) - n_electrons,
               lambda c: 2 * (6 * c * t2 - 6 * c * c * t3), c0)
    return c


@dataclass
class LNVResult:
    E: float
    Omega: float
    N: float
    mu: float
    alpha: float
    dE: float
    converged: bool
    status: int
    beta: float = 0.0
    c: tuple = ()


@dataclass
class LNVState:
    S: Matrix
    H: Matrix
    Z: Matrix
    L: Matrix
    n_electrons: float
    mode: int
    mu: float
    tol_E: float
    PX: Pattern
    PZG: Pattern
    prec: int = 0                      # product precision: F64, F32 or BF16
    n: int = 0
    E_prev: float = float("nan")
    D_prev: Optional[Matrix] = None
    g_prev: Optional[Matrix] = None
    Mg_prev: Optional[Matrix] = None
    history: list = field(default_factory=list)


def lnv_init(S: Matrix, H: Matrix, Z: Matrix, l_pattern: Pattern, n_electrons: float,
             mode: int = CANONICAL, mu: float = 0.0, tol_E: float = 1e-8,
             L0: Optional[Matrix] = None, prec: int = F64) -> LNVState:
    """Set up the minimisation.  Without L0 the start is L0 = c mask_L(Z), c from
    the cubic N(c Z) = N_e (t_m = Tr[(Z S)^m], T = Z S exact on P(r_Z + r_S))."""
    r_x = l_pattern.cutoff + max(S.pattern.cutoff, H.pattern.cutoff)
    PX = derived_pattern(l_pattern, r_x)
    PZG = derived_pattern(l_pattern, Z.pattern.cutoff + l_pattern.cutoff)
    if L0 is None:
        PT = derived_pattern(Z.pattern, Z.pattern.cutoff + S.pattern.cutoff)
        T = product(Z, S, PT)
        T2 = product(T, T, PT)
        t2 = trace_product(T, T)
        t3 = trace_product(T2, T)
        c = lnv_initial_scale(S.nrows, n_electrons, t2, t3)
        Zl = mask_copy(Z, l_pattern)
        L = Matrix(l_pattern, S.b, c * Zl.blocks)
    else:
        L = mask_copy(L0, l_pattern)
    return LNVState(S=S, H=H, Z=Z, L=L, n_electrons=n_electrons, mode=mode, mu=mu,
                    tol_E=tol_E, PX=PX, PZG=PZG, prec=prec)


def lnv_restart(st: LNVState, prec: int) -> None:
    """Keep L, clear the conjugate-gradient history, switch the product precision
    (the FP64 refinement after a low-precision stage)."""
    st.prec = prec
    st.n = 0
    st.E_prev = float("nan")
    st.D_prev = st.g_prev = st.Mg_prev = None


def _precondition(st: LNVState, G: Matrix) -> Matrix:
    """M(G) = sym(mask_L((Z G) Z)): the S^-1-contravariant form of a gradient."""
    ZG = product(st.Z, G, st.PZG, st.prec)
    return symmetrize(product(ZG, st.Z, st.L.pattern, st.prec))


def lnv_energy_terms(st: LNVState):
    """X = L S, Y = L H, W = mask(X X), U = mask(Y X) on P_X and E, N from traces."""
    PX, pr = st.PX, st.prec
    X = product(st.L, st.S, PX, pr)
    Y = product(st.L, st.H, PX, pr)
    W = product(X, X, PX, pr)
    U = product(Y, X, PX, pr)
    E = 2.0 * (3.0 * trace_product(X, Y) - 2.0 * trace_product(W, Y))
    N = 2.0 * (3.0 * trace_product(X, X) - 2.0 * trace_product(W, X))
    return X, Y, W, U, E, N


def lnv_gradients(st: LNVState, X, W, U):
    """G_E = 2[3(HX + (HX)^T) - 2(HW + (HW)^T + S U)], G_N = 12 (S X - S W), on P_L, symmetrised.

    These are dE/dL and dN/dL for E = 2 Tr[(3LSL - 2LSLSL) H], N = 2 Tr[(3LSL - 2LSLSL) S].
    """
    PL, pr = st.L.pattern, st.prec
    HX = product(st.H, X, PL, pr)
    HW = product(st.H, W, PL, pr)
    SU = product(st.S, U, PL, pr)
    SX = product(st.S, X, PL, pr)
    SW = product(st.S, W, PL, pr)
    HXt, HWt = transpose(HX), transpose(HW)
    GE = 6.0 * (HX.blocks + HXt.blocks) - 4.0 * (HW.blocks + HWt.blocks) - 4.0 * SU.blocks
    GN = 12.0 * (SX.blocks - SW.blocks)
    return symmetrize(Matrix(PL, st.L.b, GE)), symmetrize(Matrix(PL, st.L.b, GN))


def lnv_step(st: LNVState) -> LNVResult:
    """One LNV conjugate-gradient iteration with an exact cubic line search."""
    PL, b = st.L.pattern, st.L.b
    X, Y, W, U, E, N = lnv_energy_terms(st)
    if not (math.isfinite(E) and math.isfinite(N)):
        return LNVResult(E, float("nan"), N, st.mu, 0.0, float("nan"), False, ENONFINITE)
    GE, GN = lnv_gradients(st, X, W, U)
    PE, PN = _precondition(st, GE), _precondition(st, GN)
    gn_pn = dot(GN, PN)
    # G_N vanishes exactly only at an idempotent L; then N is stationary and the
    # projection and correction are skipped, keeping the previous mu
    canonical = st.mode == CANONICAL and gn_pn > 0.0
    mu = dot(GN, PE) / gn_pn if canonical else st.mu
    g = Matrix(PL, b, GE.blocks - mu * GN.blocks)
    Mg = Matrix(PL, b, PE.blocks - mu * PN.blocks)
    R = Matrix(PL, b, -Mg.blocks)
    beta = 0.0
    if st.n > 0 and st.n % 50 != 0 and st.g_prev is not None:
        den = dot(st.g_prev, st.Mg_prev)
        beta = max(0.0, dot(g, Matrix(PL, b, Mg.blocks - st.Mg_prev.blocks)) / den)
    D = Matrix(PL, b, R.blocks + beta * st.D_prev.blocks) if beta != 0.0 else R.copy()
    if dot(g, D) >= 0.0:
        beta = 0.0
        D = R.copy()
    if canonical:
        D = Matrix(PL, b, D.blocks - (dot(GN, D) / gn_pn) * PN.blocks)

    # exact line search along L + a D: X(a) = X + a X_D, Y(a) = Y + a Y_D
    PX, pr = st.PX, st.prec
    XD = product(D, st.S, PX, pr)
    YD = product(D, st.H, PX, pr)
    Q = product(XD, XD, PX, pr)
    X1 = Matrix(PX, b, X.blocks + XD.blocks)
    W1 = product(X1, X1, PX, pr)
    M1 = Matrix(PX, b, W1.blocks - W.blocks - Q.blocks)   # X XD + XD X
    tp = trace_product
    f = [tp(X, Y), tp(XD, Y) + tp(X, YD), tp(XD, YD), 0.0]
    h = [tp(X, X), 2.0 * tp(X, XD), tp(XD, XD), 0.0]
    gg = [tp(W, Y), tp(M1, Y) + tp(W, YD), tp(Q, Y) + tp(M1, YD), tp(Q, YD)]
    kk = [tp(W, X), tp(M1, X) + tp(W, XD), tp(Q, X) + tp(M1, XD), tp(Q, XD)]
    e = [2.0 * (3.0 * f[m] - 2.0 * gg[m]) for m in range(4)]
    nn = [2.0 * (3.0 * h[m] - 2.0 * kk[m]) for m in range(4)]
    c = [e[m] - mu * nn[m] for m in range(4)]
    disc = c[2] * c[2] - 3.0 * c[1] * c[3]
    status = OK
    if not (disc >= 0.0):
        status = ERUNAWAY
    else:
        den = c[2] + math.sqrt(disc)
        if not (den > 0.0):
            status = ERUNAWAY
    dE = E - st.E_prev if st.n > 0 else float("nan")
    Omega = E - mu * N
    if status != OK:
        return LNVResult(E, Omega, N, mu, 0.0, dE, False, status, beta, tuple(c))
    a = -c[1] / den
    Lnew = st.L.blocks + a * D.blocks
    if canonical:
        N_a = nn[0] + a * (nn[1] + a * (nn[2] + a * nn[3]))
        delta = (st.n_electrons - N_a) / gn_pn
        Lnew = Lnew + delta * PN.blocks
    st.L = symmetrize(Matrix(PL, b, Lnew))
    converged = st.n > 0 and abs(dE) < st.tol_E
    st.E_prev = E
    st.mu = mu
    st.D_prev, st.g_prev, st.Mg_prev = D, g, Mg
    st.n += 1
    res = LNVResult(E, Omega, N, mu, a, dE, converged, OK, beta, tuple(c))
    st.history.append(res)
    return res


def lnv_solve(st: LNVState, stages) -> dict:
    """A precision schedule, stage by stage: lnv_step in stage precision until
    |dE| < tol (tol > 0), or E fails to decrease (stop_on_rise), or max_iter steps;
    later stages keep L and restart the conjugate gradients."""
    out = dict(status=OK, converged=False, iterations=[], E=float("nan"), N=float("nan"))
    for s, (prec, max_iter, tol, rise) in enumerate(stages):
        if s > 0:
            lnv_restart(st, prec)
        else:
            st.prec = prec
        stop, it = False, 0
        while it < max_iter and not stop:
            r = lnv_step(st)
            it += 1
            out["E"], out["N"] = r.E, r.N
            if r.status != OK:
                out["status"] = r.status
                out["iterations"].append(it)
                return out
            if st.n > 1:
                if tol > 0 and abs(r.dE) < tol:
                    stop = True
                if rise and not (r.dE < 0.0):
                    stop = True
        out["iterations"].append(it)
        if s == len(stages) - 1:
            out["converged"] = stop or tol <= 0
    return out


def idempotency_error(st: LNVState) -> float:
    """e = ||mask_X(KS KS) - KS||_F / ||KS||_F with KS = 3W - 2 mask_X(W X) on P_X.

    KS = 3(LS)^2 - 2(LS)^3; for an idempotent K (K S K = K) KS is a projector.
    Products in FP64 whatever the state's precision."""
    PX = st.PX
    X = product(st.L, st.S, PX)
    W = product(X, X, PX)
    WX = product(W, X, PX)
    KS = Matrix(PX, st.L.b, 3.0 * W.blocks - 2.0 * WX.blocks)
    KS2 = product(KS, KS, PX)
    num = float(np.linalg.norm((KS2.blocks - KS.blocks).ravel()))
    return num / float(np.linalg.norm(KS.blocks.ravel()))


def density_matrix(st: LNVState, pattern: Pattern) -> Matrix:
    """K = 3 LSL - 2 LSLSL on `pattern`; exact when the pattern range is at most r_S
    (W = X X is held on P(r_L + r_S) and W L must reach r_L beyond it)."""
    X = product(st.L, st.S, st.PX)
    W = product(X, X, st.PX)
    K = product(X, st.L, pattern)
    K2 = product(W, st.L, pattern)
    return Matrix(pattern, st.L.b, 3.0 * K.blocks - 2.0 * K2.blocks)


# ---------------------------------------------------------------------------
# Forces from the converged density matrix
# ---------------------------------------------------------------------------
def lnv_chemical_potential(st: LNVState) -> float:
    """mu = <G_N, M(G_E)> / <G_N, M(G_N)> at the current L (the canonical definition)."""
    X, Y, W, U, E, N = lnv_energy_terms(st)
    GE, GN = lnv_gradients(st, X, W, U)
    PE, PN = _precondition(st, GE), _precondition(st, GN)
    return dot(GN, PE) / dot(GN, PN)


def lnv_forces(st: LNVState, dS: List[Matrix], dH: List[Matrix], mu: Optional[float] = None) -> np.ndarray:
    """Forces F_I = -d Omega / d R_I at a converged L, Omega = E - mu (N - N_e).

    The paper lists forces with the solver's next capabilities; this is the
    standard derivative of the density-matrix functional.  At a stationary L
    (G_E = mu G_N on P_L) dE/dR = dOmega/dR at fixed L.  With K = 3LSL - 2LSLSL,
    H' = H - mu S and the energy-density matrix Q = 3 L H' L - 2 (LSL H' L + L H' LSL),
        dOmega = 2 Tr[K dH] + 2 Tr[(Q - mu K) dS].
    dS and dH hold, for every block (i, j) of S and H, d(block)/dR_j per Cartesian
    direction (d/dR_i is its negative; blocks of an atom with itself do not move),
    so with K, Q symmetric the derivative with respect to atom I collapses onto its
    row:  F_I^c = 4 sum_{j != I} <K_Ij, dH^c_Ij> + <(Q - mu K)_Ij, dS^c_Ij>  (elementwise).
    Needs r_S == r_H.  Q is exact on P_S: L H' on P_X = P(r_L + r_S), M = L H' L
    on P(r_X + r_S) (all that X M reads for outputs on P_S), X M with X = L S
    masked to P_S.  mu: the chemical potential to use (default: from the current
    gradients, lnv_chemical_potential).
    """
    S, H, L = st.S, st.H, st.L
    PS = S.pattern
    assert abs(PS.cutoff - H.pattern.cutoff) < 1e-12, "forces need the S and H patterns equal"
    b = S.b
    if mu is None:
        mu = lnv_chemical_potential(st)
    K = density_matrix(st, PS)
    Hp = Matrix(PS, b, H.blocks - mu * S.blocks)
    X = product(L, S, st.PX)
    LH = product(L, Hp, st.PX)
    PM = derived_pattern(L.pattern, st.PX.cutoff + PS.cutoff)
    M = product(LH, L, PM)
    XM = product(X, M, PS)
    Q = Matrix(PS, b, 3.0 * mask_copy(M, PS).blocks - 2.0 * (XM.blocks + transpose(XM).blocks))
    Wt = Q.blocks - mu * K.blocks
    rows = PS.rows()
    off = rows != PS.cols
    F = np.zeros((PS.natoms, 3))
    for c in range(3):
        per_block = (np.einsum("nab,nab->n", K.blocks, dH[c].blocks) +
                     np.einsum("nab,nab->n", Wt, dS[c].blocks))
        np.add.at(F[:, c], rows[off], 4.0 * per_block[off])
    return F


# ---------------------------------------------------------------------------
# Contraction to support functions
# ---------------------------------------------------------------------------
def contract(M: Matrix, coef: np.ndarray) -> Matrix:
    """Blocks of M in a basis of bc support functions per atom, each a combination of
    the atom's own b orbitals with coefficients coef[i] (b x bc):  M'_ij = C_i^T M_ij C_j
    on the same pattern: single-site support functions, the on-site equivalent of
    multi-site support functions that the paper lists among its development
    priorities for PAO basis sets (Development Priorities)."""
    coef = np.asarray(coef, np.float64)
    P = M.pattern
    rows, cols = P.rows(), P.cols
    out = np.einsum("nab,nac,ncd->nbd", coef[rows], M.blocks, coef[cols])
    return Matrix(P, coef.shape[2], out)
