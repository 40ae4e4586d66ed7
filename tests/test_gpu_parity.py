"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded inputs.

Tolerances: patterns and flop counts bit-exact; single products, traces and
inner products within 1e-12 of the result scale (only the summation order
differs); Hotelling after 10 steps and LNV after 20 iterations within 1e-10
relative.
"""
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


@pytest.fixture(scope="module")
def ctx(bsm):
    return bsm.Context(0)


def gpat(bsm, ctx, pos, box, r, b):
    return bsm.Pattern(ctx, torch.tensor(pos, dtype=torch.float64, device=ctx.device), box, r, b)


def gmat(bsm, P, blocks):
    return bsm.Matrix(P, torch.tensor(np.ascontiguousarray(blocks), dtype=torch.float64, device=P.ctx.device))


def host(M):
    torch.cuda.synchronize()
    return M.blocks.cpu().numpy()


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


SYSTEMS = {
    "si64": lambda: synth.si64_b4(),
    "si64_disp": lambda: synth.make_system("d", 2, 4, synth.SMALL_CUTOFFS, 3, displacement_sigma=0.2),
    "ortho_2x3x4": lambda: synth.make_system("o", (2, 3, 4), 4, synth.SMALL_CUTOFFS, 4, displacement_sigma=0.05),
    "si256_disp": lambda: synth.make_system("d2", (4, 4, 2), 4, synth.SMALL_CUTOFFS, 5, displacement_sigma=0.1),
    "si216_disp": lambda: synth.make_system("d3", (3, 3, 3), 4, synth.SMALL_CUTOFFS, 6, displacement_sigma=0.1),
}


# ------------------------------------------------------------------ patterns
@pytest.mark.parametrize("name,cutoffs", [("si64", [3.0, 6.0, 8.0, 10.0, 14.0, 30.0]),
                                          ("si64_disp", [4.0, 6.0, 7.3]),
                                          ("ortho_2x3x4", [2.5, 6.0, 9.0, 16.0]),
                                          ("si256_disp", [6.0, 8.0, 12.0])])
def test_pattern_bitexact(bsm, ctx, name, cutoffs):
    s = SYSTEMS[name]()
    for r in cutoffs:
        say(f"pattern {name} r={r}")
        P = gpat(bsm, ctx, s.positions, s.box, r, 4)
        rp, cols = P.to_host()
        Po = O.create_pattern(s.positions, s.box, r)
        assert np.array_equal(rp, Po.rowptr) and np.array_equal(cols, Po.cols), (name, r)
        assert P.max_row == int(np.diff(Po.rowptr).max())


@pytest.mark.parametrize("r", [6.0, 10.0, 16.0])
def test_pattern_4096_bitexact(bsm, ctx, r):
    pos, box, _ = synth.diamond_positions((8, 8, 8))
    say(f"pattern 4096 r={r}")
    P = gpat(bsm, ctx, pos, box, r, 9)
    rp, cols = P.to_host()
    Po = O.create_pattern(pos, box, r)
    assert np.array_equal(rp, Po.rowptr) and np.array_equal(cols, Po.cols)


def test_pattern_single_atom(bsm, ctx):
    P = gpat(bsm, ctx, np.array([[1.0, 2.0, 3.0]]), (5.0, 5.0, 5.0), 2.0, 9)
    rp, cols = P.to_host()
    assert list(rp) == [0, 1] and list(cols) == [0]


def test_pattern_rejects_bad_input(bsm, ctx):
    pos = np.zeros((4, 3))
    with pytest.raises(bsm.BSMError) as e:
        gpat(bsm, ctx, pos, (5.0, 5.0, 5.0), -1.0, 4)
    assert e.value.code == bsm.EINVAL
    pos[1, 0] = np.nan
    with pytest.raises(bsm.BSMError) as e:
        gpat(bsm, ctx, pos, (5.0, 5.0, 5.0), 2.0, 4)
    assert e.value.code == bsm.EINVAL


def test_pattern_row_cap(bsm, ctx):
    """Rows are sorted in LDS, so a row holds at most 8192 blocks: a cutoff past every
    minimum-image distance gives rows of all atoms; 8192 atoms build (every row full,
    columns in order), 8193 are refused before any row is written, and the context
    stays usable."""
    rng = np.random.default_rng(8192)
    box = (40.0, 40.0, 40.0)
    pos = rng.uniform(0.0, 40.0, (8193, 3))
    say("pattern row cap: 8192 atoms, full rows")
    P = gpat(bsm, ctx, pos[:8192], box, 100.0, 1)
    rp, cols = P.to_host()
    assert P.max_row == 8192
    assert np.array_equal(rp, np.arange(8193, dtype=np.int64) * 8192)
    full = np.arange(8192)
    for i in (0, 4095, 8191):
        assert np.array_equal(cols[rp[i]:rp[i + 1]], full)
    del P
    say("pattern row cap: 8193 atoms refused")
    with pytest.raises(bsm.BSMError) as e:
        gpat(bsm, ctx, pos, box, 100.0, 1)
    assert e.value.code == bsm.EINVAL and "8192" in str(e.value)
    P = gpat(bsm, ctx, pos[:64], box, 12.0, 4)
    Po = O.create_pattern(pos[:64], box, 12.0)
    rp, cols = P.to_host()
    assert np.array_equal(rp, Po.rowptr) and np.array_equal(cols, Po.cols)


# ------------------------------------------------------------------ products
PRODUCT_CASES = [(6, 6, 8), (8, 6, 5), (3, 8, 6), (6, 8, 14), (12, 12, 12), (8, 8, 3)]


@pytest.mark.parametrize("b", [1, 4, 9, 16])
def test_product_parity(bsm, ctx, b):
    s = SYSTEMS["si256_disp"]()
    cut = sorted({r for case in PRODUCT_CASES for r in case})
    gp = {r: gpat(bsm, ctx, s.positions, s.box, float(r), b) for r in cut}
    op = {r: O.create_pattern(s.positions, s.box, float(r)) for r in cut}
    for n, (ra, rb, rc) in enumerate(PRODUCT_CASES):
        say(f"product b={b} P{ra} x P{rb} -> P{rc}")
        a = synth.random_blocks(op[ra].nnz, b, 10 + n)
        bb = synth.random_blocks(op[rb].nnz, b, 20 + n)
        c0 = synth.random_blocks(op[rc].nnz, b, 30 + n)
        A, B, C = gmat(bsm, gp[ra], a), gmat(bsm, gp[rb], bb), gmat(bsm, gp[rc], c0)
        bsm.multiply_truncate(0.75, A, B, -0.5, C)
        Co = O.Matrix(op[rc], b, c0.copy())
        O.multiply_truncate(0.75, O.Matrix(op[ra], b, a), O.Matrix(op[rb], b, bb), -0.5, Co)
        assert rel_err(host(C), Co.blocks) < 1e-12
        # algorithmic flop count: 2 b^3 per block triple, bit-exact
        tri = O.count_triples(op[ra], op[rb], op[rc]).sum()
        assert bsm.product_flops(gp[ra], gp[rb], gp[rc]) == 2.0 * b ** 3 * tri


@pytest.mark.parametrize("variant,rows,system", [(0, 2, "si256_disp"), (0, 4, "si256_disp"), (0, 8, "si256_disp"),
                                                  (1, 2, "si256_disp"), (1, 4, "si256_disp"), (2, 0, "si256_disp"),
                                                  (2, 0, "si216_disp"), (3, 4, "si256_disp"), (3, 2, "si216_disp"),
                                                  (4, 4, "si216_disp"), (4, 2, "si256_disp"), (4, 8, "si216_disp"),
                                                  (5, 8, "si216_disp"), (5, 4, "si256_disp"), (5, 2, "si216_disp"),
                                                  (6, 8, "si216_disp"), (6, 4, "si256_disp")])
@pytest.mark.parametrize("b", [4, 9])
def test_product_kernel_variants(bsm, b, variant, rows, system):
    """Every product kernel variant and rows-per-wave choice gives the oracle's result
    (216 atoms: the last 16-row workgroup tile is half empty; variant 6, the FP64
    matrix-core tiles, runs for b = 9 and falls back to the ring for b = 4)."""
    ctx = bsm.Context(0)
    ctx.set_product_variant(variant)
    ctx.set_rows_per_wave(rows)
    s = SYSTEMS[system]()
    say(f"product variant={variant} rows={rows} b={b}")
    gp = {r: gpat(bsm, ctx, s.positions, s.box, float(r), b) for r in (6, 8, 14)}
    op = {r: O.create_pattern(s.positions, s.box, float(r)) for r in (6, 8, 14)}
    for n, (ra, rb, rc) in enumerate([(6, 8, 14), (14, 8, 6), (8, 8, 8)]):
        a = synth.random_blocks(op[ra].nnz, b, 40 + n)
        bb = synth.random_blocks(op[rb].nnz, b, 50 + n)
        c0 = synth.random_blocks(op[rc].nnz, b, 60 + n)
        A, B, C = gmat(bsm, gp[ra], a), gmat(bsm, gp[rb], bb), gmat(bsm, gp[rc], c0)
        bsm.multiply_truncate(1.25, A, B, 0.5, C)
        Co = O.Matrix(op[rc], b, c0.copy())
        O.multiply_truncate(1.25, O.Matrix(op[ra], b, a), O.Matrix(op[rb], b, bb), 0.5, Co)
        assert rel_err(host(C), Co.blocks) < 1e-12, (ra, rb, rc)
    ctx.close()


@pytest.mark.parametrize("variant,rows", [(1, 4), (4, 4), (4, 8), (4, 2), (2, 0), (5, 8), (5, 4), (6, 8), (6, 4)])
@pytest.mark.parametrize("b", [4, 9])
def test_product_degenerate_cases(bsm, b, variant, rows):
    """One atom (one tile, one entry padded to two); diagonal-only operands into a
    wide output pattern (most tiles have no entries and only apply beta)."""
    ctx = bsm.Context(0)
    ctx.set_product_variant(variant)
    ctx.set_rows_per_wave(rows)
    say(f"degenerate products variant={variant} rows={rows} b={b}")
    one = np.array([[1.0, 2.0, 3.0]])
    P1 = gpat(bsm, ctx, one, (5.0, 5.0, 5.0), 2.0, b)
    a = synth.random_blocks(1, b, 5)
    bb = synth.random_blocks(1, b, 6)
    c0 = synth.random_blocks(1, b, 7)
    C = gmat(bsm, P1, c0)
    bsm.multiply_truncate(2.0, gmat(bsm, P1, a), gmat(bsm, P1, bb), 0.5, C)
    assert rel_err(host(C), 2.0 * a @ bb + 0.5 * c0) < 1e-14
    s = SYSTEMS["si216_disp"]()
    gd, g6 = gpat(bsm, ctx, s.positions, s.box, 1.0, b), gpat(bsm, ctx, s.positions, s.box, 6.0, b)
    od, o6 = O.create_pattern(s.positions, s.box, 1.0), O.create_pattern(s.positions, s.box, 6.0)
    assert od.nnz == len(s.positions)
    a = synth.random_blocks(od.nnz, b, 8)
    bb = synth.random_blocks(od.nnz, b, 9)
    c0 = synth.random_blocks(o6.nnz, b, 10)
    C = gmat(bsm, g6, c0)
    bsm.multiply_truncate(1.5, gmat(bsm, gd, a), gmat(bsm, gd, bb), -0.25, C)
    Co = O.Matrix(o6, b, c0.copy())
    O.multiply_truncate(1.5, O.Matrix(od, b, a), O.Matrix(od, b, bb), -0.25, Co)
    assert rel_err(host(C), Co.blocks) < 1e-13
    # and the FP32 path on the same degenerate product
    C = gmat(bsm, g6, c0)
    bsm.multiply_truncate_prec(bsm.F32, 1.5, gmat(bsm, gd, a), gmat(bsm, gd, bb), -0.25, C)
    Co = O.Matrix(o6, b, c0.copy())
    O.multiply_truncate_mixed(1, 1.5, O.Matrix(od, b, a), O.Matrix(od, b, bb), -0.25, Co)
    assert rel_err(host(C), Co.blocks) < 1e-14
    ctx.close()


@pytest.mark.parametrize("variant,rows", [(4, 8), (4, 4), (3, 2), (1, 4), (2, 0), (0, 2), (5, 8)])
@pytest.mark.parametrize("b", [4, 9])
def test_product_column_orders_agree(bsm, b, variant, rows):
    """Tiles over ascending columns (order 0) and over columns grouped by the rows
    that hold outputs in them (order 1, the default) cover the same output blocks:
    FP64 and FP32 products are equal element by element (the nonzero terms of each
    element are summed in the same ascending k order), and both match the oracle;
    BF16 on the matrix cores matches the oracle under both orders.  216 atoms: the 16-row workgroup tiles end half empty."""
    s = SYSTEMS["si216_disp"]()
    op = {r: O.create_pattern(s.positions, s.box, float(r)) for r in (6, 8, 14)}
    cases = [(6, 8, 14), (14, 8, 6), (8, 14, 8)]
    data = [(synth.random_blocks(op[ra].nnz, b, 110 + n), synth.random_blocks(op[rb].nnz, b, 120 + n),
             synth.random_blocks(op[rc].nnz, b, 130 + n)) for n, (ra, rb, rc) in enumerate(cases)]
    out = {}
    mfma = b == 9 and variant in (3, 4, 5) and rows in (4, 8)   # BF16 on the matrix cores
    precs = (bsm.F64, bsm.F32, bsm.BF16) if mfma else (bsm.F64, bsm.F32)
    for order in (0, 1):
        ctx = bsm.Context(0)
        ctx.set_product_variant(variant)
        ctx.set_rows_per_wave(rows)
        ctx.set_column_order(order)
        say(f"column order={order} variant={variant} rows={rows} b={b}")
        gp = {r: gpat(bsm, ctx, s.positions, s.box, float(r), b) for r in (6, 8, 14)}
        for n, (ra, rb, rc) in enumerate(cases):
            a, bb, c0 = data[n]
            for prec in precs:
                C = gmat(bsm, gp[rc], c0)
                bsm.multiply_truncate_prec(prec, 1.25, gmat(bsm, gp[ra], a), gmat(bsm, gp[rb], bb), 0.5, C)
                out[order, n, prec] = host(C)
        ctx.close()
    if mfma:   # matrix cores: entries paired differently, so compared with the oracle only
        for order in (0, 1):
            for n, (ra, rb, rc) in enumerate(cases):
                a, bb, c0 = data[n]
                Co = O.Matrix(op[rc], b, c0.copy())
                O.multiply_truncate_mixed(2, 1.25, O.Matrix(op[ra], b, a), O.Matrix(op[rb], b, bb), 0.5, Co)
                assert rel_err(out[order, n, bsm.BF16], Co.blocks) < 2e-6, (order, ra, rb, rc)
    for n, (ra, rb, rc) in enumerate(cases):
        a, bb, c0 = data[n]
        for prec in (bsm.F64, bsm.F32):
            assert np.array_equal(out[0, n, prec], out[1, n, prec]), (n, prec)
            Co = O.Matrix(op[rc], b, c0.copy())
            if prec == bsm.F64:
                O.multiply_truncate(1.25, O.Matrix(op[ra], b, a), O.Matrix(op[rb], b, bb), 0.5, Co)
                assert rel_err(out[1, n, prec], Co.blocks) < 1e-12, (ra, rb, rc)
            else:
                O.multiply_truncate_mixed(1, 1.25, O.Matrix(op[ra], b, a), O.Matrix(op[rb], b, bb), 0.5, Co)
                assert rel_err(out[1, n, prec], Co.blocks) < 1e-14, (ra, rb, rc)


@pytest.mark.parametrize("b", [4, 9])
def test_product_variants_bitwise_equal(bsm, b):
    """Every FP64 kernel variant and tile height sums each output element's terms in
    ascending (k, m) order with fused multiply-adds, so all give the same bits."""
    s = SYSTEMS["si216_disp"]()
    op = {r: O.create_pattern(s.positions, s.box, float(r)) for r in (6, 8, 14)}
    a = synth.random_blocks(op[14].nnz, b, 140)
    bb = synth.random_blocks(op[8].nnz, b, 141)
    c0 = synth.random_blocks(op[8].nnz, b, 142)
    ref = None
    # (3, 8): the 8-row ring with 64-bit addresses, which variant 4 also runs for operands past 4 GB
    for variant, rows in [(4, 8), (0, 2), (0, 8), (1, 4), (2, 0), (3, 4), (3, 2), (3, 8), (4, 4), (5, 8), (5, 4)]:
        ctx = bsm.Context(0)
        ctx.set_product_variant(variant)
        ctx.set_rows_per_wave(rows)
        say(f"bitwise variant={variant} rows={rows} b={b}")
        gp = {r: gpat(bsm, ctx, s.positions, s.box, float(r), b) for r in (8, 14)}
        C = gmat(bsm, gp[8], c0)
        bsm.multiply_truncate(0.75, gmat(bsm, gp[14], a), gmat(bsm, gp[8], bb), -0.5, C)
        got = host(C)
        ctx.close()
        if ref is None:
            ref = got
            Co = O.Matrix(op[8], b, c0.copy())
            O.multiply_truncate(0.75, O.Matrix(op[14], b, a), O.Matrix(op[8], b, bb), -0.5, Co)
            assert rel_err(ref, Co.blocks) < 1e-12
        else:
            assert np.array_equal(got, ref), (variant, rows)


@pytest.mark.parametrize("b", [4, 9])
@pytest.mark.parametrize("cutoffs", [(14, 8, 8), (6, 8, 14), (8, 8, 8)])
def test_product_pair_equals_two_products(bsm, b, cutoffs):
    """bsm_multiply_truncate_pair (C = A B, C2 = A2 B sharing B's copies in one launch) gives
    the bits of two bsm_multiply_truncate calls, which match the oracle; with a kernel variant
    that has no paired tiles it runs as two launches; A2 or C2 off A's or C's pattern is refused."""
    ra, rb, rc = cutoffs
    s = SYSTEMS["si216_disp"]()
    op = {r: O.create_pattern(s.positions, s.box, float(r)) for r in set(cutoffs)}
    a = synth.random_blocks(op[ra].nnz, b, 150)
    a2 = synth.random_blocks(op[ra].nnz, b, 151)
    bb = synth.random_blocks(op[rb].nnz, b, 152)
    c0 = synth.random_blocks(op[rc].nnz, b, 153)
    c20 = synth.random_blocks(op[rc].nnz, b, 154)
    got = {}
    for variant in (-1, 1):
        ctx = bsm.Context(0)
        ctx.set_product_variant(variant)
        say(f"pair product b={b} P{ra} x P{rb} -> P{rc}, variant {variant}")
        gp = {r: gpat(bsm, ctx, s.positions, s.box, float(r), b) for r in set(cutoffs)}
        A, A2, B = gmat(bsm, gp[ra], a), gmat(bsm, gp[ra], a2), gmat(bsm, gp[rb], bb)
        C, C2 = gmat(bsm, gp[rc], c0), gmat(bsm, gp[rc], c20)
        bsm.multiply_truncate_pair(1.25, A, A2, B, -0.5, C, C2)
        S1, S2 = gmat(bsm, gp[rc], c0), gmat(bsm, gp[rc], c20)
        bsm.multiply_truncate(1.25, A, B, -0.5, S1)
        bsm.multiply_truncate(1.25, A2, B, -0.5, S2)
        assert np.array_equal(host(C), host(S1)) and np.array_equal(host(C2), host(S2)), variant
        got[variant] = (host(C), host(C2))
        if variant == -1:
            other = gpat(bsm, ctx, s.positions, s.box, float(ra), b)   # same cutoff, another pattern
            with pytest.raises(bsm.BSMError) as e:
                bsm.multiply_truncate_pair(1.0, A, gmat(bsm, other, a2), B, 0.0, C, C2)
            assert e.value.code == bsm.EPATTERN
            with pytest.raises(bsm.BSMError) as e:
                bsm.multiply_truncate_pair(1.0, A, A2, B, 0.0, C, C)
            assert e.value.code == bsm.EINVAL
        ctx.close()
    for (x, x0, m) in ((got[-1][0], c0, a), (got[-1][1], c20, a2)):
        Co = O.Matrix(op[rc], b, x0.copy())
        O.multiply_truncate(1.25, O.Matrix(op[ra], b, m), O.Matrix(op[rb], b, bb), -0.5, Co)
        assert rel_err(x, Co.blocks) < 1e-12


@pytest.mark.parametrize("b", [4, 9])
@pytest.mark.parametrize("cutoffs", [(8, 6, 14), (14, 8, 8), (8, 8, 8)])
def test_product_pair_a_equals_two_products(bsm, b, cutoffs):
    """bsm_multiply_truncate_pair_a (C = A B, C2 = A B2 sharing A's copies, on a transposed plan)
    gives the bits of two bsm_multiply_truncate calls, which match the oracle; with a kernel
    variant that has no paired tiles it runs as two launches; B2 off B's pattern is refused."""
    ra, rb, rc = cutoffs
    s = SYSTEMS["si216_disp"]()
    op = {r: O.create_pattern(s.positions, s.box, float(r)) for r in set(cutoffs)}
    a = synth.random_blocks(op[ra].nnz, b, 160)
    bb = synth.random_blocks(op[rb].nnz, b, 161)
    bb2 = synth.random_blocks(op[rb].nnz, b, 162)
    c0 = synth.random_blocks(op[rc].nnz, b, 163)
    c20 = synth.random_blocks(op[rc].nnz, b, 164)
    got = None
    for variant in (-1, 1):
        ctx = bsm.Context(0)
        ctx.set_product_variant(variant)
        say(f"pair_a product b={b} P{ra} x P{rb} -> P{rc}, variant {variant}")
        gp = {r: gpat(bsm, ctx, s.positions, s.box, float(r), b) for r in set(cutoffs)}
        A, B, B2 = gmat(bsm, gp[ra], a), gmat(bsm, gp[rb], bb), gmat(bsm, gp[rb], bb2)
        C, C2 = gmat(bsm, gp[rc], c0), gmat(bsm, gp[rc], c20)
        bsm.multiply_truncate_pair_a(1.25, A, B, B2, -0.5, C, C2)
        S1, S2 = gmat(bsm, gp[rc], c0), gmat(bsm, gp[rc], c20)
        bsm.multiply_truncate(1.25, A, B, -0.5, S1)
        bsm.multiply_truncate(1.25, A, B2, -0.5, S2)
        assert np.array_equal(host(C), host(S1)) and np.array_equal(host(C2), host(S2)), variant
        if variant == -1:
            got = (host(C), host(C2))
            other = gpat(bsm, ctx, s.positions, s.box, float(rb), b)
            with pytest.raises(bsm.BSMError) as e:
                bsm.multiply_truncate_pair_a(1.0, A, B, gmat(bsm, other, bb2), 0.0, C, C2)
            assert e.value.code == bsm.EPATTERN
        ctx.close()
    for (x, x0, m) in ((got[0], c0, bb), (got[1], c20, bb2)):
        Co = O.Matrix(op[rc], b, x0.copy())
        O.multiply_truncate(1.25, O.Matrix(op[ra], b, a), O.Matrix(op[rb], b, m), -0.5, Co)
        assert rel_err(x, Co.blocks) < 1e-12


@pytest.mark.parametrize("b", [4, 9])
def test_product_pairs_degenerate(bsm, b):
    """Pairs on one atom (one tile, one entry padded to two) and on diagonal-only operands into a
    wide output pattern (most tiles have no entries and only apply beta): equal bits to single
    products, for both the shared-right and the shared-left pair."""
    ctx = bsm.Context(0)
    one = np.array([[1.0, 2.0, 3.0]])
    s = SYSTEMS["si216_disp"]()
    cases = [(gpat(bsm, ctx, one, (5.0, 5.0, 5.0), 2.0, b),) * 3]
    gd, g6 = gpat(bsm, ctx, s.positions, s.box, 1.0, b), gpat(bsm, ctx, s.positions, s.box, 6.0, b)
    cases.append((gd, gd, g6))
    for n, (pa, pb, pc) in enumerate(cases):
        say(f"degenerate pairs b={b} case {n}")
        rnd = lambda P, seed: gmat(bsm, P, synth.random_blocks(P.nnzb, b, seed))
        A, A2, B, B2 = rnd(pa, 10 + n), rnd(pa, 20 + n), rnd(pb, 30 + n), rnd(pb, 40 + n)
        c0, c20 = synth.random_blocks(pc.nnzb, b, 50 + n), synth.random_blocks(pc.nnzb, b, 60 + n)
        C, C2, S1, S2 = gmat(bsm, pc, c0), gmat(bsm, pc, c20), gmat(bsm, pc, c0), gmat(bsm, pc, c20)
        bsm.multiply_truncate_pair(1.5, A, A2, B, -0.25, C, C2)
        bsm.multiply_truncate(1.5, A, B, -0.25, S1)
        bsm.multiply_truncate(1.5, A2, B, -0.25, S2)
        assert np.array_equal(host(C), host(S1)) and np.array_equal(host(C2), host(S2))
        C, C2, S1, S2 = gmat(bsm, pc, c0), gmat(bsm, pc, c20), gmat(bsm, pc, c0), gmat(bsm, pc, c20)
        bsm.multiply_truncate_pair_a(1.5, A, B, B2, -0.25, C, C2)
        bsm.multiply_truncate(1.5, A, B, -0.25, S1)
        bsm.multiply_truncate(1.5, A, B2, -0.25, S2)
        assert np.array_equal(host(C), host(S1)) and np.array_equal(host(C2), host(S2))
    ctx.close()


def test_product_pair_at_4096_atoms(bsm):
    """The paired launch on the 16 A x 16 A -> 16 A class of the 4096-atom, b = 9 system (the
    pair LNV uses for W = X X and U = Y X): equal bits to two single products."""
    pos, box, _ = synth.diamond_positions((8, 8, 8))
    ctx = bsm.Context(0)
    P = gpat(bsm, ctx, pos, box, 16.0, 9)
    g = torch.Generator(device=ctx.device)
    g.manual_seed(5)
    mk = lambda: bsm.Matrix(P, torch.rand((P.nnzb, 9, 9), dtype=torch.float64, device=ctx.device, generator=g) - 0.5)
    X, Y = mk(), mk()
    W, U, W1, U1 = bsm.Matrix(P), bsm.Matrix(P), bsm.Matrix(P), bsm.Matrix(P)
    say("pair product 4096 atoms b=9, 16 A")
    bsm.multiply_truncate_pair(1.0, X, Y, X, 0.0, W, U)
    bsm.multiply_truncate(1.0, X, X, 0.0, W1)
    bsm.multiply_truncate(1.0, Y, X, 0.0, U1)
    torch.cuda.synchronize()
    assert torch.equal(W.blocks, W1.blocks) and torch.equal(U.blocks, U1.blocks)
    ctx.close()


@pytest.mark.parametrize("rows", [8, 4])
@pytest.mark.parametrize("b", [4, 9])
def test_transposed_plans_agree(bsm, b, rows):
    """Products planned as C = (B^T A^T)^T (blocks read transposed, C's blocks written
    at the transposed slots) equal the direct products element by element in FP64
    and FP32 (the same terms in the same order), on classes where A and B lie on
    different patterns; both match the oracle.  BF16 on the matrix cores keeps
    direct plans."""
    s = SYSTEMS["si216_disp"]()
    op = {r: O.create_pattern(s.positions, s.box, float(r)) for r in (6, 8, 14)}
    cases = [(14, 8, 6), (14, 6, 8), (8, 14, 8), (6, 8, 14), (14, 8, 14)]
    data = [(synth.random_blocks(op[ra].nnz, b, 150 + n), synth.random_blocks(op[rb].nnz, b, 160 + n),
             synth.random_blocks(op[rc].nnz, b, 170 + n)) for n, (ra, rb, rc) in enumerate(cases)]
    precs = (bsm.F64, bsm.F32, bsm.BF16) if b == 9 else (bsm.F64, bsm.F32)
    out = {}
    for mode in (0, 2):
        ctx = bsm.Context(0)
        ctx.set_rows_per_wave(rows)
        ctx.set_transposed_plans(mode)
        say(f"transposed plans mode={mode} rows={rows} b={b}")
        gp = {r: gpat(bsm, ctx, s.positions, s.box, float(r), b) for r in (6, 8, 14)}
        for n, (ra, rb, rc) in enumerate(cases):
            a, bb, c0 = data[n]
            for prec in precs:
                C = gmat(bsm, gp[rc], c0)
                bsm.multiply_truncate_prec(prec, 1.25, gmat(bsm, gp[ra], a), gmat(bsm, gp[rb], bb), -0.5, C)
                out[mode, n, prec] = host(C)
        ctx.close()
    for n, (ra, rb, rc) in enumerate(cases):
        a, bb, c0 = data[n]
        for prec in precs:
            if prec != bsm.BF16:
                assert np.array_equal(out[0, n, prec], out[2, n, prec]), (ra, rb, rc, prec)
            Co = O.Matrix(op[rc], b, c0.copy())
            if prec == bsm.F64:
                O.multiply_truncate(1.25, O.Matrix(op[ra], b, a), O.Matrix(op[rb], b, bb), -0.5, Co)
                tol = 1e-12
            else:
                O.multiply_truncate_mixed(prec, 1.25, O.Matrix(op[ra], b, a), O.Matrix(op[rb], b, bb), -0.5, Co)
                tol = 2e-6 if prec == bsm.BF16 else 1e-14
            for mode in (0, 2):
                assert rel_err(out[mode, n, prec], Co.blocks) < tol, (mode, ra, rb, rc, prec)


@pytest.mark.parametrize("b", [4, 9])
def test_transposed_plan_beta_zero_ignores_nan(bsm, b):
    """A transposed plan with beta = 0 writes every C block (at the transposed slots)
    without reading C: a NaN-filled C comes out finite and equal to the direct plan's."""
    s = SYSTEMS["si216_disp"]()
    op = {r: O.create_pattern(s.positions, s.box, float(r)) for r in (6, 8, 14)}
    a = synth.random_blocks(op[14].nnz, b, 180)
    bb = synth.random_blocks(op[6].nnz, b, 181)
    out = {}
    for mode in (0, 2):
        ctx = bsm.Context(0)
        ctx.set_transposed_plans(mode)
        gp = {r: gpat(bsm, ctx, s.positions, s.box, float(r), b) for r in (6, 8, 14)}
        C = gmat(bsm, gp[8], np.full((op[8].nnz, b, b), np.nan))
        bsm.multiply_truncate(1.0, gmat(bsm, gp[14], a), gmat(bsm, gp[6], bb), 0.0, C)
        out[mode] = host(C)
        ctx.close()
    assert np.isfinite(out[2]).all()
    assert np.array_equal(out[0], out[2])


def test_transposed_plans_reject_bad_mode(bsm, ctx):
    with pytest.raises(bsm.BSMError):
        ctx.set_transposed_plans(3)


def test_column_order_rejects_bad_value(bsm, ctx):
    with pytest.raises(bsm.BSMError):
        ctx.set_column_order(2)


def test_product_beta_zero_ignores_nan_and_is_deterministic(bsm, ctx):
    s = SYSTEMS["si64"]()
    P6, P8 = (gpat(bsm, ctx, s.positions, s.box, r, 4) for r in (6.0, 8.0))
    o6, o8 = (O.create_pattern(s.positions, s.box, r) for r in (6.0, 8.0))
    a = synth.random_blocks(o6.nnz, 4, 1)
    A, B = gmat(bsm, P6, a), gmat(bsm, P6, a[::-1])
    C = gmat(bsm, P8, np.full((o8.nnz, 4, 4), np.nan))
    bsm.multiply_truncate(1.0, A, B, 0.0, C)
    first = host(C).copy()
    assert np.isfinite(first).all()
    for _ in range(3):
        bsm.multiply_truncate(1.0, A, B, 0.0, C)
        assert np.array_equal(host(C), first)
    want = O.product(O.Matrix(o6, 4, a), O.Matrix(o6, 4, a[::-1].copy()), o8)
    assert rel_err(first, want.blocks) < 1e-13


def test_product_errors(bsm, ctx):
    s = SYSTEMS["si64"]()
    P4 = gpat(bsm, ctx, s.positions, s.box, 6.0, 4)
    P9 = gpat(bsm, ctx, s.positions, s.box, 6.0, 9)
    A4, A9 = bsm.Matrix(P4), bsm.Matrix(P9)
    with pytest.raises(bsm.BSMError) as e:
        bsm.multiply_truncate(1.0, A4, A9, 0.0, bsm.Matrix(P4))
    assert e.value.code == bsm.EPATTERN
    with pytest.raises(bsm.BSMError) as e:
        bsm.multiply_truncate(1.0, A4, A4, 0.0, A4)
    assert e.value.code == bsm.EINVAL


def test_fill_blocks_outside_pattern(bsm, ctx):
    s = SYSTEMS["si64"]()
    P3 = gpat(bsm, ctx, s.positions, s.box, 3.0, 4)
    M = bsm.Matrix(P3)
    with pytest.raises(bsm.BSMError) as e:
        bsm.fill_blocks(M, s.S.rows, s.S.cols, s.S.blocks)   # S reaches 6 A
    assert e.value.code == bsm.EPATTERN


# ------------------------------------------------------------------ reductions and elementwise
@pytest.mark.parametrize("ra,rb", [(6, 6), (6, 8), (3, 12), (8, 5)])
def test_trace_parity(bsm, ctx, ra, rb):
    s = SYSTEMS["si256_disp"]()
    say(f"trace P{ra} . P{rb}")
    ga, gb = gpat(bsm, ctx, s.positions, s.box, float(ra), 9), gpat(bsm, ctx, s.positions, s.box, float(rb), 9)
    oa, ob = O.create_pattern(s.positions, s.box, float(ra)), O.create_pattern(s.positions, s.box, float(rb))
    a, b = synth.random_blocks(oa.nnz, 9, 3), synth.random_blocks(ob.nnz, 9, 4)
    want = O.trace_product(O.Matrix(oa, 9, a), O.Matrix(ob, 9, b))
    scale = np.sqrt((a ** 2).sum() * (b ** 2).sum())
    got = bsm.trace_product(gmat(bsm, ga, a), gmat(bsm, gb, b))
    assert abs(got - want) <= 1e-13 * scale
    assert bsm.trace_product(gmat(bsm, ga, a), gmat(bsm, gb, b)) == got   # bitwise reproducible


def test_elementwise_parity(bsm, ctx):
    s = SYSTEMS["si256_disp"]()
    g6, g8 = gpat(bsm, ctx, s.positions, s.box, 6.0, 9), gpat(bsm, ctx, s.positions, s.box, 8.0, 9)
    o6, o8 = O.create_pattern(s.positions, s.box, 6.0), O.create_pattern(s.positions, s.box, 8.0)
    a, b = synth.random_blocks(o8.nnz, 9, 5), synth.random_blocks(o8.nnz, 9, 6)
    X, Y = gmat(bsm, g8, a), gmat(bsm, g8, b)
    assert abs(bsm.dot(X, Y) - O.dot(O.Matrix(o8, 9, a), O.Matrix(o8, 9, b))) <= 1e-12 * np.abs(a * b).sum()
    bsm.axpby(2.5, X, -0.5, Y)
    np.testing.assert_allclose(host(Y), 2.5 * a - 0.5 * b, rtol=1e-15, atol=1e-15)
    bsm.symmetrize(X)
    np.testing.assert_array_equal(host(X), O.symmetrize(O.Matrix(o8, 9, a)).blocks)
    M6 = bsm.Matrix(g6)
    bsm.mask_copy(X, M6)
    np.testing.assert_array_equal(host(M6), O.mask_copy(O.symmetrize(O.Matrix(o8, 9, a)), o6).blocks)
    M8 = bsm.Matrix(g8)
    bsm.mask_copy(M6, M8)    # into a larger pattern: zero fill
    np.testing.assert_array_equal(host(M8), O.mask_copy(O.Matrix(o6, 9, host(M6)), o8).blocks)
    bsm.set_identity(M8, 0.25)
    np.testing.assert_array_equal(host(M8), O.identity(o8, 9, 0.25).blocks)


# ------------------------------------------------------------------ Hotelling
def _load_SH(bsm, ctx, s):
    P6 = gpat(bsm, ctx, s.positions, s.box, s.cutoffs["S"], s.b)
    S, H = bsm.Matrix(P6), bsm.Matrix(P6)
    bsm.fill_blocks(S, s.S.rows, s.S.cols, s.S.blocks)
    bsm.fill_blocks(H, s.H.rows, s.H.cols, s.H.blocks)
    o6 = O.create_pattern(s.positions, s.box, s.cutoffs["S"])
    oS = O.from_blocks(o6, s.b, s.S.rows, s.S.cols, s.S.blocks)
    oH = O.from_blocks(o6, s.b, s.H.rows, s.H.cols, s.H.blocks)
    assert np.array_equal(host(S), oS.blocks) and np.array_equal(host(H), oH.blocks)
    return S, H, oS, oH


@pytest.mark.parametrize("b", [4, 9])
def test_hotelling_parity_small(bsm, ctx, b):
    s = synth.make_system("h", 2, b, synth.SMALL_CUTOFFS, 2205)
    say(f"hotelling 64 atoms b={b}")
    S, _, oS, _ = _load_SH(bsm, ctx, s)
    PZ = gpat(bsm, ctx, s.positions, s.box, 8.0, b)
    Z = bsm.Matrix(PZ)
    r = bsm.hotelling_inverse(S, Z, max_iter=10, tol=0.0)
    ro = O.hotelling_inverse(oS, O.create_pattern(s.positions, s.box, 8.0), max_iter=10, tol=0.0)
    assert r.status == ro.status == 0 and r.iterations == ro.iterations
    assert r.alpha == pytest.approx(ro.alpha, rel=1e-14)   # row sums in another order
    np.testing.assert_allclose(r.residuals, ro.residuals, rtol=1e-10, atol=1e-12)
    assert rel_err(host(Z), ro.Z.blocks) < 1e-10


def test_hotelling_untruncated_converges_to_inverse(bsm, ctx):
    s = synth.si64_b4()
    S, _, oS, _ = _load_SH(bsm, ctx, s)
    Z = bsm.Matrix(gpat(bsm, ctx, s.positions, s.box, 30.0, 4))
    r = bsm.hotelling_inverse(S, Z, max_iter=60, tol=1e-12)
    assert r.status == 0
    Zd = O.Matrix(O.create_pattern(s.positions, s.box, 30.0), 4, host(Z)).to_dense()
    np.testing.assert_allclose(Zd, np.linalg.inv(oS.to_dense()), atol=1e-12)


def test_hotelling_failures(bsm, ctx):
    bad = synth.make_system("bad", 2, 4, synth.SMALL_CUTOFFS, 2205, s_amp=3.0)
    S, _, oS, _ = _load_SH(bsm, ctx, bad)
    Z = bsm.Matrix(gpat(bsm, ctx, bad.positions, bad.box, 8.0, 4))
    r = bsm.hotelling_inverse(S, Z, max_iter=200, tol=1e-12, raise_on_error=False)
    assert r.status == bsm.EDIVERGED
    s = synth.si64_b4()
    S, _, _, _ = _load_SH(bsm, ctx, s)
    S.blocks[7, 1, 2] = float("nan")
    r = bsm.hotelling_inverse(S, Z, max_iter=5, tol=1e-12, raise_on_error=False)
    assert r.status == bsm.ENONFINITE


# ------------------------------------------------------------------ LNV
def _lnv_pair(bsm, ctx, s, mode=0, mu=0.0, rl=None, rz=None, hot_iter=10, tol_E=1e-8):
    rl = s.cutoffs["L"] if rl is None else rl
    rz = s.cutoffs["Z"] if rz is None else rz
    S, H, oS, oH = _load_SH(bsm, ctx, s)
    Z = bsm.Matrix(gpat(bsm, ctx, s.positions, s.box, rz, s.b))
    bsm.hotelling_inverse(S, Z, max_iter=hot_iter, tol=0.0)
    L = bsm.Matrix(gpat(bsm, ctx, s.positions, s.box, rl, s.b))
    g = bsm.LNV(S, H, Z, L, s.n_electrons, mode=mode, mu=mu, tol_E=tol_E)
    oz = O.hotelling_inverse(oS, O.create_pattern(s.positions, s.box, rz), max_iter=hot_iter, tol=0.0).Z
    st = O.lnv_init(oS, oH, oz, O.create_pattern(s.positions, s.box, rl), s.n_electrons, mode=mode, mu=mu,
                    tol_E=tol_E)
    assert rel_err(host(L), st.L.blocks) < 1e-12
    return g, L, st


@pytest.mark.parametrize("b", [4, 9])
def test_lnv_parity_20_iterations(bsm, ctx, b):
    s = synth.make_system("l", 2, b, synth.SMALL_CUTOFFS, 2205)
    say(f"lnv 64 atoms b={b}")
    g, L, st = _lnv_pair(bsm, ctx, s)
    for it in range(20):
        rg, ro = g.step(), O.lnv_step(st)
        assert rg.status == ro.status == 0
        assert abs(rg.E - ro.E) <= 1e-10 * abs(ro.E), (it, rg.E, ro.E)
        assert abs(rg.N - ro.N) <= 1e-10 * abs(ro.N)
        if it < 6:   # later, c1 is a small difference of O(10) traces and alpha carries its rounding
            assert abs(rg.alpha - ro.alpha) <= 1e-6 * abs(ro.alpha), (it, rg.alpha, ro.alpha)
    Lg, Lo = host(L), st.L.blocks
    assert np.linalg.norm(Lg - Lo) / np.linalg.norm(Lo) < 1e-8
    assert rg.product_flops > 0


def test_lnv_bond_projector_closed_form(bsm, ctx):
    s = synth.make_system("bond", 2, 9, synth.SMALL_CUTOFFS, 5, s_amp=0.0, h_random=False)
    g, L, st = _lnv_pair(bsm, ctx, s, tol_E=1e-12)
    for _ in range(60):
        r = g.step()
        if r.converged:
            break
    assert abs(r.E - (-4 * 64 * synth.T_BOND)) < 1e-9


def test_lnv_grand_and_runaway(bsm, ctx):
    s = synth.si64_b4()
    g, L, st = _lnv_pair(bsm, ctx, s, mode=1, mu=0.0)
    om = [g.step().Omega for _ in range(8)]
    assert all(b < a for a, b in zip(om, om[1:]))
    # L = 2 Z with mu far below the spectrum: no minimum along the line
    S, H, oS, oH = _load_SH(bsm, ctx, s)
    Z = bsm.Matrix(gpat(bsm, ctx, s.positions, s.box, 8.0, 4))
    bsm.hotelling_inverse(S, Z, max_iter=10, tol=0.0)
    L = bsm.Matrix(Z.pattern, 2.0 * Z.blocks.clone())
    g = bsm.LNV(S, H, Z, L, s.n_electrons, mode=1, mu=-10.0, init_from_z=False)
    assert g.step().status == bsm.ERUNAWAY


# ------------------------------------------------------------------ 4096 atoms, 9 orbitals
def test_w_class_product_4096_sampled(bsm, ctx):
    """The 16 A x 16 A -> 16 A product at full size, in the launch the benchmark
    times; sampled output rows checked against the oracle."""
    pos, box, _ = synth.diamond_positions((8, 8, 8))
    say("W-class 4096 atoms b=9: patterns")
    P16 = gpat(bsm, ctx, pos, box, 16.0, 9)
    o16 = O.create_pattern(pos, box, 16.0)
    rng = np.random.default_rng(2205)
    x = rng.uniform(-1, 1, (o16.nnz, 9, 9))
    y = rng.uniform(-1, 1, (o16.nnz, 9, 9))
    say("W-class 4096 atoms b=9: GPU product")
    X, Y = gmat(bsm, P16, x), gmat(bsm, P16, y)
    C = bsm.Matrix(P16)
    bsm.multiply_truncate(1.0, X, Y, 0.0, C)
    assert bsm.product_flops(P16, P16, P16) == 2.0 * 729 * O.count_triples(o16, o16, o16).sum()
    g = host(C)
    rows = [0, 1, 7, 1000, 2047, 4095]
    say("W-class 4096 atoms b=9: oracle rows", rows)
    Co = O.Matrix(o16, 9)
    for r in rows:
        O.multiply_truncate(1.0, O.Matrix(o16, 9, x), O.Matrix(o16, 9, y), 0.0, Co, r, r + 1)
        sl = slice(o16.rowptr[r], o16.rowptr[r + 1])
        assert rel_err(g[sl], Co.blocks[sl]) < 1e-12, r


def test_w_class_product_past_4gb_sampled(bsm, ctx):
    """8192 atoms at 16 A: each operand holds 4.5 GB, past what the default kernel's
    buffer copies address, so the same tiles run with 64-bit copy addresses; sampled
    output rows against the oracle, and the flop count against the oracle's triples."""
    pos, box, _ = synth.diamond_positions((16, 8, 8))
    say("16 A product, 8192 atoms b=9: patterns")
    P16 = gpat(bsm, ctx, pos, box, 16.0, 9)
    o16 = O.create_pattern(pos, box, 16.0)
    assert o16.nnz * 81 * 8 > 0xFFFFF000
    rng = np.random.default_rng(2206)
    x = rng.uniform(-1, 1, (o16.nnz, 9, 9))
    y = rng.uniform(-1, 1, (o16.nnz, 9, 9))
    say("16 A product, 8192 atoms b=9: GPU product")
    X, Y = gmat(bsm, P16, x), gmat(bsm, P16, y)
    C = bsm.Matrix(P16)
    bsm.multiply_truncate(1.0, X, Y, 0.0, C)
    g = host(C)
    del X, Y, C
    assert bsm.product_flops(P16, P16, P16) == 2.0 * 729 * O.count_triples(o16, o16, o16).sum()
    rows = [0, 4095, 4096, 8191]
    say("16 A product, 8192 atoms b=9: oracle rows", rows)
    Co = O.Matrix(o16, 9)
    for r in rows:
        O.multiply_truncate(1.0, O.Matrix(o16, 9, x), O.Matrix(o16, 9, y), 0.0, Co, r, r + 1)
        sl = slice(o16.rowptr[r], o16.rowptr[r + 1])
        assert rel_err(g[sl], Co.blocks[sl]) < 1e-12, r


# ------------------------------------------------------------------ mixed precision and diagnostics
@pytest.mark.parametrize("prec,b,variant,rows", [(1, 4, -1, 0), (1, 9, -1, 0), (1, 9, -1, 4), (2, 4, -1, 0),
                                                (2, 9, 1, 0), (2, 9, -1, 0), (2, 9, -1, 4), (2, 9, -1, 8),
                                                (1, 9, 5, 0), (1, 4, 5, 0), (2, 4, 5, 0), (2, 9, 5, 0)])
def test_mixed_product_parity(bsm, prec, b, variant, rows):
    """FP32 / BF16-rounded operands, FP32 accumulation.  VALU kernels: the oracle's
    result up to the FP64 epilogue (same rounding, same accumulation order).  BF16
    with b = 9 on the matrix cores (the default): the same BF16 inputs and exact
    FP32 products, summed in the matrix core's order, so the sums differ from the
    oracle's FMA chain by FP32 rounding only: checked against the oracle at 2e-6 of
    the result scale (a few hundred terms per element, FP32 unit roundoff 6e-8).
    4- and 8-row tiles both run BF16 on the matrix cores when A and B share a pattern;
    products of two patterns take the BF16-rounded VALU ring (the oracle's bits)."""
    ctx = bsm.Context(0)
    ctx.set_product_variant(variant)
    ctx.set_rows_per_wave(rows)
    mfma = prec == 2 and b == 9 and variant in (-1, 5)
    s = SYSTEMS["si256_disp"]()
    say(f"mixed product prec={prec} b={b} variant={variant} rows={rows}")
    gp = {r: gpat(bsm, ctx, s.positions, s.box, float(r), b) for r in (6, 8, 14)}
    op = {r: O.create_pattern(s.positions, s.box, float(r)) for r in (6, 8, 14)}
    for n, (ra, rb, rc) in enumerate([(6, 8, 14), (14, 8, 6), (8, 8, 14)]):
        a = synth.random_blocks(op[ra].nnz, b, 70 + n)
        bb = synth.random_blocks(op[rb].nnz, b, 80 + n)
        c0 = synth.random_blocks(op[rc].nnz, b, 90 + n)
        A, B, C = gmat(bsm, gp[ra], a), gmat(bsm, gp[rb], bb), gmat(bsm, gp[rc], c0)
        bsm.multiply_truncate_prec(prec, 0.5, A, B, 0.25, C)
        Co = O.Matrix(op[rc], b, c0.copy())
        O.multiply_truncate_mixed(prec, 0.5, O.Matrix(op[ra], b, a), O.Matrix(op[rb], b, bb), 0.25, Co)
        err = rel_err(host(C), Co.blocks)
        say(f"   P{ra} x P{rb} -> P{rc}: {err:.3e}")
        assert err < (2e-6 if mfma and ra == rb else 1e-14)
    ctx.close()


@pytest.mark.parametrize("b", [4, 9])
def test_idempotency_error_parity(bsm, ctx, b):
    s = synth.make_system("l", 2, b, synth.SMALL_CUTOFFS, 2205)
    g, L, st = _lnv_pair(bsm, ctx, s)
    for _ in range(6):
        g.step()
        O.lnv_step(st)
    eg, eo = g.idempotency_error(), O.idempotency_error(st)
    assert eg == pytest.approx(eo, rel=1e-8)
    assert g.step().E == pytest.approx(O.lnv_step(st).E, rel=1e-10)   # the diagnostic left the state intact


@pytest.mark.parametrize("b", [4, 9])
def test_mixed_schedule_reaches_fp64_energy(bsm, ctx, b):
    """BF16 then FP32 products (FP64 traces), then 3 FP64 steps: the energy of the
    FP64 oracle's converged solve to better than 1e-6 Ha/atom, on GPU and oracle alike."""
    s = synth.make_system("l", 2, b, synth.SMALL_CUTOFFS, 2205)
    say(f"mixed schedule b={b}")
    g, L, st = _lnv_pair(bsm, ctx, s)
    o_ref = O.lnv_init(st.S, st.H, st.Z, st.L.pattern, s.n_electrons, tol_E=1e-11)
    for _ in range(100):
        if O.lnv_step(o_ref).converged:
            break
    E_ref = o_ref.E_prev
    stages = [(2, 30, 0.0, True), (1, 60, 1e-6, True), (0, 3, 0.0, False)]
    rg = g.solve(stages)
    ro = O.lnv_solve(st, stages)
    assert rg["status"] == 0 and ro["status"] == 0 and rg["converged"]
    assert abs(rg["E"] - E_ref) / 64 < 1e-6 and abs(ro["E"] - E_ref) / 64 < 1e-6
    assert abs(rg["E"] - ro["E"]) / 64 < 1e-6
    assert rg["product_flops"] > 0


# ------------------------------------------------------------------ batched persistent launch
def _batch_case(bsm, ctx, seed):
    """Uneven small systems, b = 4 and 9, three product shapes."""
    specs = [((2, 2, 2), 4), ((2, 2, 3), 9), ((2, 3, 3), 4), ((3, 3, 3), 9), ((2, 2, 2), 9), ((2, 3, 2), 4)]
    out = []
    for n, (cells, b) in enumerate(specs):
        pos, box, _ = synth.diamond_positions(cells)
        ra, rb, rc = [(6, 8, 14), (8, 8, 8), (14, 6, 10)][n % 3]
        gp = {r: gpat(bsm, ctx, pos, box, float(r), b) for r in {ra, rb, rc}}
        op = {r: O.create_pattern(pos, box, float(r)) for r in {ra, rb, rc}}
        a = synth.random_blocks(op[ra].nnz, b, seed + 3 * n)
        bb = synth.random_blocks(op[rb].nnz, b, seed + 3 * n + 1)
        out.append(dict(b=b, A=gmat(bsm, gp[ra], a), B=gmat(bsm, gp[rb], bb), C=bsm.Matrix(gp[rc]),
                        C1=bsm.Matrix(gp[rc]), oA=O.Matrix(op[ra], b, a), oB=O.Matrix(op[rb], b, bb), oPC=op[rc]))
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_separate_products(bsm, ctx, prec):
    case = _batch_case(bsm, ctx, 100 + prec)
    say(f"batch prec={prec}: {len(case)} products")
    batch = bsm.Batch(ctx, [(c["A"], c["B"], c["C"]) for c in case], alpha=1.5, beta=0.0, precision=prec)
    for mode in (bsm.BATCH_ONE_LAUNCH, bsm.BATCH_PER_B, bsm.BATCH_SEPARATE):
        for order in (0, 1, 2):
            for queues in (1, 8):
                for c in case:
                    c["C"].blocks.fill_(float("nan"))
                batch.run(order=order, waves_per_cu=8, queues=queues, mode=mode)
                for c in case:
                    bsm.multiply_truncate_prec(prec, 1.5, c["A"], c["B"], 0.0, c["C1"])
                    assert torch.equal(c["C"].blocks, c["C1"].blocks), (mode, order, queues, c["b"])
    for c in case:
        Co = O.Matrix(c["oPC"], c["b"])
        O.multiply_truncate_mixed(prec, 1.5, c["oA"], c["oB"], 0.0, Co)
        assert rel_err(host(c["C"]), Co.blocks) < 1e-13
    cfg, ms = batch.tune(reps=1)
    assert cfg["queues"] in (1, 8) and cfg["waves_per_cu"] in (4, 8, 16) and ms > 0
    assert cfg["mode"] in (bsm.BATCH_ONE_LAUNCH, bsm.BATCH_PER_B, bsm.BATCH_SEPARATE)
    before = [c["C"].blocks.clone() for c in case]
    batch.run()
    for c, x in zip(case, before):
        assert torch.equal(c["C"].blocks, x)
    assert batch.flops == sum(bsm.product_flops(c["A"].pattern, c["B"].pattern, c["C"].pattern) for c in case)
    batch.close()
