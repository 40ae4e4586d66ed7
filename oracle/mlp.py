"""FP64 CPU oracle of the learned initial guess: pair descriptors and a 3-layer MLP.

TEST INFRASTRUCTURE ONLY.  Plain numpy definitions that the HIP descriptor and
network kernels must reproduce; only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library.

The paper names machine-learned methods as one of the directions for the code
(Development Priorities) but fixes no model; this network is an extension
built on the method.  It predicts corrections to the method's own starting
points from local geometry:

    L0 = c mask_L(Z) + dL,      Z0 = alpha I + dZ,

where c mask_L(Z) and alpha I are the plain starts of the LNV minimisation and
the Hotelling iteration, and dL, dZ are predicted block by block from a
descriptor of each atom pair.  A network whose last layer is zero therefore
reproduces the plain starts exactly.

Descriptor of the pair (i, j), r = minimum-image vector from atom i to atom j,
d = |r|, r_c the cutoff of the pattern it is evaluated on (32 values):

    r / r_c (3), d / r_c, (d / r_c)^2, exp(-d / 1.5 A), s_i, s_j,
    rhat . e_i[a] (a = 0..3), rhat . e_j[a] (a = 0..3),
    10 (l_i[a] - d0) (a = 0..3), 10 (l_j[a] - d0) (a = 0..3),
    10 c_i (3), 10 c_j (3), 0, 0

with rhat = r / d (0 on the diagonal), lengths in Angstrom.  s_i = +1 or -1 is
the sublattice of atom i, e_i[a] and l_i[a] the direction and length of its
bond along hybrid a, and c_i the mean of the vectors to its four nearest
neighbours (zero on the ideal lattice), all read from those neighbours
(atom_frames); d0 = a sqrt(3) / 4 is the ideal bond length, a = 5.43 A.  The
last two features measure the local strain that displacements cause.

Network (parameters as one flat FP32 array, weights stored input-major):
    h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3,
    W1: D x H, W2: H x H, W3: H x M, with D = 32, H = width, M = b^2.
Loss over a minibatch of n samples: (1 / 2n) sum_s sum_o (y_so - t_so)^2.
Optimiser: Adam (Kingma and Ba, ICLR 2015, Algorithm 1) with bias correction.
"""
from __future__ import annotations

import dataclasses

import numpy as np

TETRA = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) / np.sqrt(3.0)
DESC_DIM = 32
DECAY = 1.5   # Angstrom, the decay length of the off-site overlap
BOND0 = 5.43 * np.sqrt(3.0) / 4.0   # ideal Si-Si bond length, Angstrom


def min_image(pos: np.ndarray, box: np.ndarray, i, j) -> np.ndarray:
    d = pos[j] - pos[i]
    return d - box * np.rint(d / box)


# Overlap-weighted neighbour count of an atom of the ideal diamond lattice within
# RHO_CUTOFF: the textbook coordination shells inside 6 A (4 at a sqrt(3)/4, 12 at
# a/sqrt(2), 12 at a sqrt(11)/4, 6 at a, 12 at a sqrt(19)/4; the next, 24 at
# a sqrt(27)/4 = 7.05 A, lies outside), each weighted by exp(-d / DECAY).
RHO_CUTOFF = 6.0
RHO0 = sum(n * np.exp(-5.43 * np.sqrt(q) / 4.0 / DECAY) for q, n in ((3, 4), (8, 12), (11, 12), (16, 6), (19, 12)))


def atom_frames(pos: np.ndarray, box: np.ndarray, rho_cutoff: float = RHO_CUTOFF):
    """Sublattice sign s (N,), bond directions e (N, 4, 3), bond lengths l (N, 4),
    neighbour centroid c (N, 3) and environment density rho (N,) of every atom.

    rho_i = sum over the atoms j != i with minimum-image d_ij^2 < rho_cutoff^2 of
    exp(-d_ij / DECAY), added in ascending j: a collective measure of the
    environment (how many neighbours, how close), which the pair terms alone
    do not see.

    The four nearest neighbours are found by brute force over all atoms
    (minimum image), ordered by (squared distance, index).  With v_n their unit
    vectors, s = +1 when sum_n max_a v_n . T_a >= sum_n max_a (-v_n) . T_a, else
    -1 (T_a: the tetrahedral directions of the first sublattice), e[a] is
    the v_n with the largest s v_n . T_a (first such n on ties) and l[a] the
    length of that neighbour vector; c is the mean of the four neighbour vectors.
    """
    n = len(pos)
    s = np.zeros(n)
    e = np.zeros((n, 4, 3))
    l = np.zeros((n, 4))
    c = np.zeros((n, 3))
    rho = np.zeros(n)
    for i in range(n):
        others = np.array([j for j in range(n) if j != i])
        v = min_image(pos, box, np.full(len(others), i), others)
        d2 = (v * v).sum(1)
        acc = 0.0
        for q in np.flatnonzero(d2 < rho_cutoff * rho_cutoff):   # ascending j
            acc += float(np.exp(-np.sqrt(d2[q]) / DECAY))
        rho[i] = acc
        order = np.lexsort((others, d2))[:4]
        u = v[order] / np.sqrt(d2[order])[:, None]
        dots = u @ TETRA.T                       # (4 neighbours, 4 directions)
        sA, sB = dots.max(axis=1).sum(), (-dots).max(axis=1).sum()
        s[i] = 1.0 if sA >= sB else -1.0
        for a in range(4):
            q = int(np.argmax(s[i] * dots[:, a]))
            e[i, a] = u[q]
            l[i, a] = np.sqrt(d2[order][q])
        c[i] = v[order].mean(axis=0)
    return s, e, l, c, rho


def pair_descriptors(pos: np.ndarray, box: np.ndarray, rows: np.ndarray, cols: np.ndarray,
                     cutoff: float, frames) -> np.ndarray:
    """(nnz, 32) descriptors of the pattern slots (rows[k], cols[k]), in slot order."""
    s, e, l, c, rho = frames
    r = min_image(pos, box, rows, cols)
    d = np.sqrt((r * r).sum(1))
    rhat = np.where(d[:, None] > 0, r / np.where(d > 0, d, 1.0)[:, None], 0.0)
    out = np.zeros((len(rows), DESC_DIM))
    out[:, 0:3] = r / cutoff
    out[:, 3] = d / cutoff
    out[:, 4] = (d / cutoff) ** 2
    out[:, 5] = np.exp(-d / DECAY)
    out[:, 6] = s[rows]
    out[:, 7] = s[cols]
    out[:, 8:12] = np.einsum("nc,nac->na", rhat, e[rows])
    out[:, 12:16] = np.einsum("nc,nac->na", rhat, e[cols])
    out[:, 16:20] = 10.0 * (l[rows] - BOND0)
    out[:, 20:24] = 10.0 * (l[cols] - BOND0)
    out[:, 24:27] = 10.0 * c[rows]
    out[:, 27:30] = 10.0 * c[cols]
    out[:, 30] = 10.0 * (rho[rows] - RHO0)
    out[:, 31] = 10.0 * (rho[cols] - RHO0)
    return out


@dataclasses.dataclass
class Shape:
    width: int = 128
    out_dim: int = 81
    in_dim: int = DESC_DIM

    @property
    def count(self) -> int:
        D, H, M = self.in_dim, self.width, self.out_dim
        return D * H + H + H * H + H + H * M + M


def unpack(params: np.ndarray, sh: Shape):
    D, H, M = sh.in_dim, sh.width, sh.out_dim
    p = np.asarray(params, np.float64)
    o = 0
    W1 = p[o:o + D * H].reshape(D, H); o += D * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H * M].reshape(H, M); o += H * M
    b3 = p[o:o + M]
    return W1, b1, W2, b2, W3, b3


def forward(params, sh: Shape, X: np.ndarray) -> np.ndarray:
    W1, b1, W2, b2, W3, b3 = unpack(params, sh)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    return h2 @ W3 + b3


def loss_grad(params, sh: Shape, X: np.ndarray, T: np.ndarray):
    """Loss (1 / 2n) sum (y - t)^2 and its gradient with respect to the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(params, sh)
    n = len(X)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    y = h2 @ W3 + b3
    r = y - T
    loss = 0.5 * float((r * r).sum()) / n
    dy = r / n
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    dz2 = (dy @ W3.T) * (1.0 - h2 * h2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * (1.0 - h1 * h1)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, grad


@dataclasses.dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


def adam_step(params, m, v, t: int, grad, opt: Adam):
    """One Adam update at step t (1-based); returns new (params, m, v)."""
    m = opt.beta1 * m + (1.0 - opt.beta1) * grad
    v = opt.beta2 * v + (1.0 - opt.beta2) * grad * grad
    mhat = m / (1.0 - opt.beta1 ** t)
    vhat = v / (1.0 - opt.beta2 ** t)
    return params - opt.lr * mhat / (np.sqrt(vhat) + opt.eps), m, v


def train(params, sh: Shape, X, T, perm, batch: int, epochs: int, opt: Adam):
    """Minibatch k of every epoch holds samples perm[k batch : (k + 1) batch]; one Adam
    step per minibatch.  Returns the parameters and the mean minibatch loss per epoch."""
    p = np.asarray(params, np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    t = 0
    losses = []
    n = len(perm)
    for _ in range(epochs):
        acc, nb = 0.0, 0
        for k0 in range(0, n, batch):
            idx = perm[k0:k0 + batch]
            loss, g = loss_grad(p, sh, X[idx], T[idx])
            t += 1
            p, m, v = adam_step(p, m, v, t, g, opt)
            acc += loss
            nb += 1
        losses.append(acc / nb)
    return p, losses


def targets(A: np.ndarray, B: np.ndarray, scale: float) -> np.ndarray:
    """Training targets of a pattern's blocks: (A - B) / scale, one row of b^2 per slot."""
    return ((A - B) / scale).reshape(len(A), -1)
