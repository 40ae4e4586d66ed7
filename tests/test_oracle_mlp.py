"""Pins of the MLP / descriptor oracle against facts fixed outside it:
central differences, closed-form networks, Adam's known step sizes, and
the geometry of the diamond lattice (generator's sublattice labels)."""
import numpy as np
import pytest

import synth
from oracle import mlp as M


def _rand_params(sh, seed, scale=0.3):
    return scale * np.random.default_rng(seed).standard_normal(sh.count)


def test_gradient_matches_central_differences():
    sh = M.Shape(width=8, out_dim=5, in_dim=16)
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (23, 16))
    T = rng.uniform(-1, 1, (23, 5))
    p = _rand_params(sh, 2, 0.5)
    loss, g = M.loss_grad(p, sh, X, T)
    assert loss == pytest.approx(0.5 * ((M.forward(p, sh, X) - T) ** 2).sum() / 23, rel=1e-14)
    h = 1e-5
    for k in range(sh.count):
        e = np.zeros(sh.count)
        e[k] = h
        fd = (M.loss_grad(p + e, sh, X, T)[0] - M.loss_grad(p - e, sh, X, T)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g).max()), k


def test_forward_permutation_network():
    # W1, W2 permutation matrices (not symmetric), biases 0, W3 picks the first outputs:
    # y_o = tanh(tanh(x_{q(p(o))})) with the weights read input-major.
    sh = M.Shape(width=16, out_dim=3, in_dim=16)
    p1 = np.roll(np.arange(16), 3)        # h1_o = tanh(x_{p1[o]})
    p2 = np.roll(np.arange(16), -5)       # h2_o = tanh(h1_{p2[o]})
    W1 = np.zeros((16, 16)); W1[p1, np.arange(16)] = 1.0
    W2 = np.zeros((16, 16)); W2[p2, np.arange(16)] = 1.0
    W3 = np.zeros((16, 3)); W3[np.arange(3), np.arange(3)] = 1.0
    b3 = np.array([0.5, -1.0, 2.0])
    params = np.concatenate([W1.ravel(), np.zeros(16), W2.ravel(), np.zeros(16), W3.ravel(), b3])
    X = np.random.default_rng(3).uniform(-2, 2, (7, 16))
    Y = M.forward(params, sh, X)
    for o in range(3):
        assert np.allclose(Y[:, o], np.tanh(np.tanh(X[:, p1[p2[o]]])) + b3[o], rtol=0, atol=1e-15)


def test_forward_constant_layers():
    # W1 = W2 = 0: h1 = tanh(b1), h2 = tanh(b2) for every input; y = h2 W3 + b3
    sh = M.Shape(width=4, out_dim=2, in_dim=16)
    b1 = np.arctanh(np.array([0.5, -0.5, 0.25, 0.0]))
    b2 = np.arctanh(np.array([0.1, 0.2, 0.3, 0.4]))
    W3 = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0], [2.0, -1.0]])
    params = np.concatenate([np.zeros(64), b1, np.zeros(16), b2, W3.ravel(), [0.0, 1.0]])
    Y = M.forward(params, sh, np.ones((3, 16)))
    assert np.allclose(Y, [[0.1 + 0.3 + 0.8, 0.2 + 0.3 - 0.4 + 1.0]] * 3, atol=1e-15)


def test_zero_last_layer_predicts_zero():
    sh = M.Shape(width=8, out_dim=4, in_dim=16)
    p = _rand_params(sh, 5)
    p[-(8 * 4 + 4):] = 0.0
    assert not np.any(M.forward(p, sh, np.random.default_rng(0).uniform(-1, 1, (9, 16))))


def test_adam_step_sizes():
    # bias-corrected Adam: with a constant gradient g every step moves by lr g / (|g| + eps)
    opt = M.Adam(lr=0.01)
    p = np.zeros(4)
    m = np.zeros(4); v = np.zeros(4)
    g = np.array([3.0, -0.2, 1e-3, 0.0])
    for t in range(1, 6):
        q, m, v = M.adam_step(p, m, v, t, g, opt)
        assert np.allclose(q - p, -opt.lr * g / (np.abs(g) + opt.eps), rtol=1e-12, atol=1e-18)
        p = q


def test_training_fits_a_linear_target():
    sh = M.Shape(width=16, out_dim=2, in_dim=16)
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (256, 16))
    T = np.stack([0.3 * X[:, 0] - 0.2 * X[:, 5], 0.1 * X[:, 3]], 1)
    p0 = _rand_params(sh, 6, 0.2)
    _, losses = M.train(p0, sh, X, T, np.arange(256), 64, 40, M.Adam(lr=3e-3))
    assert losses[-1] < 0.05 * losses[0]


def test_frames_on_the_ideal_lattice():
    pos, box, sub = synth.diamond_positions((2, 2, 2))
    s, e, l, c, _ = M.atom_frames(pos, box)
    assert np.array_equal(s, np.where(sub == 0, 1.0, -1.0))
    # every bond direction is exactly the sublattice's tetrahedral direction, every bond ideal
    assert np.allclose(e, s[:, None, None] * M.TETRA[None], atol=1e-12)
    assert np.allclose(l, 5.43 * np.sqrt(3) / 4, atol=1e-12) and np.allclose(c, 0.0, atol=1e-12)


def test_descriptors_of_the_ideal_lattice():
    pos, box, sub = synth.diamond_positions((2, 2, 2))
    fr = M.atom_frames(pos, box)
    n = len(pos)
    rows, cols = np.repeat(np.arange(n), n), np.tile(np.arange(n), n)
    X = M.pair_descriptors(pos, box, rows, cols, 8.0, fr)
    d = X[:, 3] * 8.0
    nn = np.abs(d - 5.43 * np.sqrt(3) / 4) < 1e-9
    assert nn.sum() == 4 * n
    # a bond lies along exactly one hybrid of each end: cosine 1 at i, -1 at j, -1/3 / +1/3 elsewhere
    ci, cj = X[nn, 8:12], X[nn, 12:16]
    assert np.allclose(np.sort(ci, 1), [[-1 / 3, -1 / 3, -1 / 3, 1]] * nn.sum(), atol=1e-12)
    assert np.allclose(np.sort(cj, 1), [[-1, 1 / 3, 1 / 3, 1 / 3]] * nn.sum(), atol=1e-12)
    assert np.all(X[nn, 6] == -X[nn, 7])                  # bonds join the two sublattices
    # the diagonal: r = 0
    dg = rows == cols
    assert np.allclose(X[dg][:, [0, 1, 2, 3, 4, 8, 9, 10, 11, 12, 13, 14, 15]], 0.0)
    assert np.allclose(X[dg, 5], 1.0)
    # reflection: (j, i) has -r, the same distance, swapped sublattices and cosine groups negated
    Xt = X.reshape(n, n, 32).transpose(1, 0, 2).reshape(-1, 32)
    off = ~dg
    assert np.allclose(Xt[off, 0:3], -X[off, 0:3], atol=1e-14)
    assert np.allclose(Xt[off, 3:6], X[off, 3:6], atol=1e-14)
    assert np.array_equal(Xt[off, 6], X[off, 7])
    assert np.allclose(Xt[off, 8:12], -X[off, 12:16], atol=1e-14)
    # no strain on the ideal lattice
    assert np.allclose(X[:, 16:30], 0.0, atol=1e-11)


def test_environment_density_of_the_ideal_lattice():
    # 3 x 3 x 3 cells (box 16.3 A): every atom sees the infinite lattice's shells inside 6 A, so
    # its density is the textbook value and the environment features vanish; a 2 x 2 x 2 cell
    # (box 10.86 A) folds the shell at a = 5.43 A onto 3 atoms and the one at a sqrt(19)/4 onto
    # fewer atoms, so there the density is lower
    pos, box, _ = synth.diamond_positions((3, 3, 3))
    fr = M.atom_frames(pos, box)
    assert np.allclose(fr[4], M.RHO0, rtol=1e-14)
    assert M.RHO0 == pytest.approx(4 * np.exp(-2.3513 / 1.5) + 12 * np.exp(-3.8396 / 1.5) + 12 * np.exp(-4.5023 / 1.5)
                                   + 6 * np.exp(-5.43 / 1.5) + 12 * np.exp(-5.9172 / 1.5), rel=1e-4)
    n = len(pos)
    X = M.pair_descriptors(pos, box, np.arange(n), np.arange(n), 8.0, fr)
    assert np.allclose(X[:, 30:32], 0.0, atol=1e-12)
    small = M.atom_frames(*synth.diamond_positions((2, 2, 2))[:2])
    assert np.all(small[4] < M.RHO0 - 0.01)
    # a displaced frame: an atom pushed toward its neighbours gains density
    sy = synth.displaced_frame(3, 4, seed=10003, sigma=0.05)
    fr2 = M.atom_frames(sy.positions, sy.box)
    assert np.abs(fr2[4] - M.RHO0).max() > 1e-3 and np.abs(fr2[4] - M.RHO0).max() < 0.5


def test_frames_of_a_displaced_frame_keep_the_sublattices():
    sy = synth.displaced_frame(2, 4, seed=10000, sigma=0.05)
    _, _, sub = synth.diamond_positions((2, 2, 2))
    s, e, l, c, _ = M.atom_frames(sy.positions, sy.box)
    assert np.array_equal(s, np.where(sub == 0, 1.0, -1.0))
    # each hybrid slot holds a different neighbour, within a few degrees of the ideal direction
    cos = np.einsum("nac,ac->na", e, M.TETRA) * s[:, None]
    assert cos.min() > 0.98
    for i in range(len(s)):
        assert len({tuple(np.round(v, 12)) for v in e[i]}) == 4
    # lengths stay within a few sigma of the ideal bond; l[a] e[a] sum to 4 c (all four used once)
    assert np.abs(l - 5.43 * np.sqrt(3) / 4).max() < 0.5
    assert np.allclose((l[:, :, None] * e).sum(1), 4.0 * c, atol=1e-12)


def test_descriptors_are_translation_invariant_and_swap_under_reflection():
    sy = synth.displaced_frame(2, 4, seed=10001, sigma=0.05)
    n = sy.natoms
    rows, cols = np.repeat(np.arange(n), n), np.tile(np.arange(n), n)
    X = M.pair_descriptors(sy.positions, sy.box, rows, cols, 8.0, M.atom_frames(sy.positions, sy.box))
    moved = np.mod(sy.positions + np.array([1.3, -2.9, 7.7]), sy.box)
    X2 = M.pair_descriptors(moved, sy.box, rows, cols, 8.0, M.atom_frames(moved, sy.box))
    assert np.allclose(X, X2, atol=1e-12)
    Xt = X.reshape(n, n, 32).transpose(1, 0, 2).reshape(-1, 32)
    assert np.allclose(Xt[:, 16:20], X[:, 20:24]) and np.allclose(Xt[:, 24:27], X[:, 27:30])
    assert np.abs(X[:, 16:30]).max() > 0.1      # displacements do show up
