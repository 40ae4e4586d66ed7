"""Oracle mixed-precision products and the idempotency diagnostic."""
import struct

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
import synth


def bf16_reference(x: float) -> float:
    """Round an FP32 value to BF16, nearest even, by integer arithmetic on its bits."""
    u = struct.unpack("<I", struct.pack("<f", np.float32(x)))[0]
    if (u & 0x7F800000) == 0x7F800000:
        return struct.unpack("<f", struct.pack("<I", (u | (0x00400000 if u & 0x7FFFFF else 0)) & 0xFFFF0000))[0]
    hi, lo = u >> 16, u & 0xFFFF
    if lo > 0x8000 or (lo == 0x8000 and hi & 1):
        hi += 1
    return struct.unpack("<f", struct.pack("<I", (hi << 16) & 0xFFFFFFFF))[0]


def test_bf16_rounding_edges():
    cases = [1.0, 1.00390625, 1.01171875, 1.005859375, -3.14159, 3.3895313892515355e38, 1e-40,
             float("inf"), -float("inf"), 65504.0, 0.0, -0.0, 2.0 ** -133]
    for x in cases:
        assert O.round_bf16(x) == bf16_reference(x) or (np.isnan(x))
    # ties to even: 1 + 2^-8 lies half-way between 1 and 1 + 2^-7 -> 1; 1 + 3*2^-8 -> 1 + 2^-6
    assert O.round_bf16(1.0 + 2 ** -8) == 1.0
    assert O.round_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert np.isnan(O.round_bf16(float("nan")))
    rng = np.random.default_rng(3)
    for x in rng.standard_normal(2000) * 10 ** rng.uniform(-30, 30, 2000):
        assert O.round_bf16(float(np.float32(x))) == bf16_reference(float(np.float32(x)))


@pytest.fixture(scope="module")
def pats():
    s = synth.make_system("d", 2, 4, synth.SMALL_CUTOFFS, 3, displacement_sigma=0.1)
    return {r: O.create_pattern(s.positions, s.box, r) for r in (5.0, 6.0, 8.0)}


@pytest.mark.parametrize("prec", [O.F32, O.BF16])
@pytest.mark.parametrize("b", [4, 9])
def test_mixed_product_vs_dense_rounded(pats, prec, b):
    A = O.Matrix(pats[6.0], b, synth.random_blocks(pats[6.0].nnz, b, 1))
    B = O.Matrix(pats[8.0], b, synth.random_blocks(pats[8.0].nnz, b, 2))
    C = O.Matrix(pats[5.0], b)
    O.multiply_truncate_mixed(prec, 1.0, A, B, 0.0, C)
    rnd = (lambda v: np.float32(v)) if prec == O.F32 else (lambda v: np.vectorize(bf16_reference)(np.float32(v)))
    Ad = np.asarray(rnd(A.to_dense()), np.float64)
    Bd = np.asarray(rnd(B.to_dense()), np.float64)
    mask = np.zeros((64, 64))
    mask[pats[5.0].rows(), pats[5.0].cols] = 1
    want = (Ad @ Bd) * np.kron(mask, np.ones((b, b)))
    # exact products of rounded inputs summed in FP64 vs the FP32 accumulation: FP32 rounding only
    err = np.abs(C.to_dense() - want).max() / np.abs(want).max()
    assert err < 64 * 2.0 ** -24
    # and the FP32 result differs from the FP64 product by the input rounding
    C64 = O.product(A, B, pats[5.0])
    rel = np.abs(C.blocks - C64.blocks).max() / np.abs(C64.blocks).max()
    assert rel < (1e-5 if prec == O.F32 else 3e-2)


def test_idempotency_error_bond_projector():
    s = synth.make_system("bond", 2, 4, synth.SMALL_CUTOFFS, 5, s_amp=0.0, h_random=False)
    P6 = O.create_pattern(s.positions, s.box, 6.0)
    S = O.from_blocks(P6, 4, s.S.rows, s.S.cols, s.S.blocks)
    H = O.from_blocks(P6, 4, s.H.rows, s.H.cols, s.H.blocks)
    PZ = O.create_pattern(s.positions, s.box, 8.0)
    Z = O.hotelling_inverse(S, PZ).Z
    st = O.lnv_init(S, H, Z, O.create_pattern(s.positions, s.box, 8.0), s.n_electrons, tol_E=1e-13)
    e0 = O.idempotency_error(st)
    for _ in range(60):
        if O.lnv_step(st).converged:
            break
    assert e0 > 1e-2 and O.idempotency_error(st) < 1e-7


def test_idempotency_error_full_cutoff_matches_dense(si64):
    P6 = O.create_pattern(si64.positions, si64.box, 6.0)
    S = O.from_blocks(P6, 4, si64.S.rows, si64.S.cols, si64.S.blocks)
    H = O.from_blocks(P6, 4, si64.H.rows, si64.H.cols, si64.H.blocks)
    PF = O.create_pattern(si64.positions, si64.box, 30.0)
    Z = O.hotelling_inverse(S, PF).Z
    st = O.lnv_init(S, H, Z, PF, si64.n_electrons)
    for _ in range(5):
        O.lnv_step(st)
    L, Sd = st.L.to_dense(), S.to_dense()
    KS = 3 * L @ Sd @ L @ Sd - 2 * L @ Sd @ L @ Sd @ L @ Sd
    want = np.linalg.norm(KS @ KS - KS) / np.linalg.norm(KS)
    assert O.idempotency_error(st) == pytest.approx(want, rel=1e-8)


@pytest.mark.slow
def test_mixed_schedule_refines_to_fp64_energy(si64):
    """Low-precision stages (BF16 to its rounding floor, then FP32) and 3 FP64 steps
    reach the FP64 minimum to better than 1e-6 Ha/atom; the low-precision stage alone
    does not (it sits at its rounding floor)."""
    P6 = O.create_pattern(si64.positions, si64.box, 6.0)
    S = O.from_blocks(P6, 4, si64.S.rows, si64.S.cols, si64.S.blocks)
    H = O.from_blocks(P6, 4, si64.H.rows, si64.H.cols, si64.H.blocks)
    PZ, PL = O.create_pattern(si64.positions, si64.box, 8.0), O.create_pattern(si64.positions, si64.box, 8.0)
    Z = O.hotelling_inverse(S, PZ).Z
    ref = O.lnv_init(S, H, Z, PL, si64.n_electrons, tol_E=1e-11)
    for _ in range(100):
        if O.lnv_step(ref).converged:
            break
    E_ref = ref.E_prev
    st = O.lnv_init(S, H, Z, PL, si64.n_electrons)
    bf = O.lnv_solve(st, [(O.BF16, 30, 0.0, True)])
    assert abs(bf["E"] - E_ref) / 64 > 1e-6
    for stages in ([(O.BF16, 30, 0.0, True), (O.F32, 60, 1e-6, True), (O.F64, 3, 0.0, False)],
                   [(O.F32, 60, 1e-6, True), (O.F64, 3, 0.0, False)]):
        st = O.lnv_init(S, H, Z, PL, si64.n_electrons)
        r = O.lnv_solve(st, stages)
        assert r["status"] == O.OK and r["converged"]
        assert abs(r["E"] - E_ref) / 64 < 1e-6, (stages, r)
