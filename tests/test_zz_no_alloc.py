"""The allocation-free trace entry point against bsm_trace_product (through the C ABI).

Two calls in a row on the same device array, the second with a smaller input
(its partial sums overwrite fewer slots of the shared scratch than the first
call left), each compared bit for bit with the allocating entry point and with
the oracle's trace at 1e-12 of the result scale.
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


def _pair(bsm, ctx, s, ra, rb, seed):
    pos = torch.tensor(s.positions, dtype=torch.float64, device=ctx.device)
    PA, PB = bsm.Pattern(ctx, pos, s.box, ra, s.b), bsm.Pattern(ctx, pos, s.box, rb, s.b)
    oa, ob = O.create_pattern(s.positions, s.box, ra), O.create_pattern(s.positions, s.box, rb)
    a = synth.random_blocks(oa.nnz, s.b, seed)
    b = synth.random_blocks(ob.nnz, s.b, seed + 1)
    A = bsm.Matrix(PA, torch.tensor(a, device=ctx.device))
    B = bsm.Matrix(PB, torch.tensor(b, device=ctx.device))
    ref = O.trace_product(O.Matrix(oa, s.b, a), O.Matrix(ob, s.b, b))
    scale = O.trace_product(O.Matrix(oa, s.b, np.abs(a)), O.Matrix(ob, s.b, np.abs(b)))   # sum of |terms|
    return A, B, ref, scale


def test_noalloc_trace_equals_allocating_trace(bsm):
    ctx = bsm.Context(0)
    out = torch.full((2,), float("nan"), dtype=torch.float64, device=ctx.device)
    big = synth.make_system("na_big", (4, 4, 4), 9, synth.BIG_CUTOFFS, 3, displacement_sigma=0.05)
    small = synth.make_system("na_small", 2, 4, synth.SMALL_CUTOFFS, 4)
    for name, s, ra, rb in [("512 atoms b=9, 10 A x 6 A", big, 10.0, 6.0), ("64 atoms b=4, 8 A x 8 A", small, 8.0, 8.0)]:
        say(f"noalloc trace: {name}")
        A, B, ref, scale = _pair(bsm, ctx, s, ra, rb, 11)
        bsm.trace_product_noalloc(A, B, out[1:])
        torch.cuda.synchronize()
        got = float(out[1].item())
        want = bsm.trace_product(A, B)
        assert got == want, (name, got, want)
        assert abs(got - ref) <= 1e-13 * scale, (name, got, ref, scale)
        assert np.isnan(out[0].item())    # nothing outside the output element was written
