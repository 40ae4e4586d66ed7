"""ctypes binding of libbsm (include/bsm.h): argument marshalling only.

Every computation runs in the HIP library; torch supplies device memory (the
caching allocator, also for the library's own scratch through the allocator
callbacks) and the stream.  Importing this module fails loudly when
libbsm.so has not been built.
"""
from __future__ import annotations

import atexit
import ctypes
import math
import os
import sys
import weakref
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsm.so")

OK, EINVAL, ENOMEM, EPATTERN, EHIP, ENONFINITE, EDIVERGED, ENOTCONV, ERUNAWAY = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
F64, F32, BF16 = 0, 1, 2
CANONICAL, GRAND = 0, 1

_NAMES = {0: "BSM_OK", -1: "BSM_EINVAL", -2: "BSM_ENOMEM", -3: "BSM_EPATTERN", -4: "BSM_EHIP",
          -5: "BSM_ENONFINITE", -6: "BSM_EDIVERGED", -7: "BSM_ENOTCONV", -8: "BSM_ERUNAWAY"}


class BSMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------- C types
c_void_p, c_int, c_int64, c_double, c_size_t = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                                ctypes.c_double, ctypes.c_size_t)
ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class _Matrix(ctypes.Structure):
    _fields_ = [("pattern", c_void_p), ("dtype", c_int), ("blocks", c_void_p)]


class _PatternInfo(ctypes.Structure):
    _fields_ = [("natoms", c_int), ("b", c_int), ("nnzb", c_int64), ("max_row", c_int),
                ("cutoff", c_double), ("box", c_double * 3), ("rowptr", c_void_p), ("cols", c_void_p),
                ("tmap", c_void_p), ("diag", c_void_p), ("pos", c_void_p)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("order", c_int), ("waves_per_cu", c_int), ("queues", c_int), ("mode", c_int)]


ORDER_BY_PRODUCT, ORDER_HEAVY_FIRST, ORDER_INTERLEAVE = 0, 1, 2
BATCH_ONE_LAUNCH, BATCH_PER_B, BATCH_SEPARATE = 0, 1, 2


class _HotParams(ctypes.Structure):
    _fields_ = [("max_iter", c_int), ("tol", c_double), ("init_given", c_int)]


class _HotResult(ctypes.Structure):
    _fields_ = [("status", c_int), ("iterations", c_int), ("alpha", c_double),
                ("residuals", ctypes.POINTER(c_double)), ("capacity", c_int), ("n_residuals", c_int),
                ("product_flops", c_double), ("start", c_int)]


class _MlpShape(ctypes.Structure):
    _fields_ = [("width", c_int), ("out_dim", c_int)]


class _Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class _TrainParams(ctypes.Structure):
    _fields_ = [("epochs", c_int), ("batch", c_int), ("opt", _Adam)]


class _GuessResult(ctypes.Structure):
    _fields_ = [("accepted", c_int), ("E_plain", c_double), ("N_plain", c_double), ("E_guess", c_double),
                ("N_guess", c_double), ("product_flops", c_double)]


class _ProductStat(ctypes.Structure):
    _fields_ = [("natoms", c_int), ("b", c_int), ("cutoff_a", c_double), ("cutoff_b", c_double),
                ("cutoff_c", c_double), ("launches", c_int64), ("flops", c_double), ("ms", c_double),
                ("variant", c_int), ("rows", c_int), ("precision", c_int), ("products", c_int)]


class _LNVParams(ctypes.Structure):
    _fields_ = [("n_electrons", c_double), ("mode", c_int), ("mu", c_double), ("tol_E", c_double),
                ("init_from_z", c_int), ("product_precision", c_int)]


MAX_STAGES = 4


class _LNVSchedule(ctypes.Structure):
    _fields_ = [("n_stages", c_int), ("precision", c_int * MAX_STAGES), ("max_iter", c_int * MAX_STAGES),
                ("tol_E", c_double * MAX_STAGES), ("stop_on_rise", c_int * MAX_STAGES)]


class _LNVSolveResult(ctypes.Structure):
    _fields_ = [("status", c_int), ("converged", c_int), ("iterations", c_int * MAX_STAGES),
                ("E", c_double), ("N", c_double), ("mu", c_double), ("product_flops", c_double)]


class _LNVResult(ctypes.Structure):
    _fields_ = [("E", c_double), ("Omega", c_double), ("N", c_double), ("mu", c_double),
                ("alpha", c_double), ("beta", c_double), ("dE", c_double), ("c", c_double * 4),
                ("converged", c_int), ("status", c_int), ("product_flops", c_double)]


EXPORTS = {
    "bsm_ctx_create": (c_int, [c_int, c_void_p, ALLOC_FN, FREE_FN, c_void_p, ctypes.POINTER(c_void_p)]),
    "bsm_ctx_destroy": (c_int, [c_void_p]),
    "bsm_ctx_set_stream": (c_int, [c_void_p, c_void_p]),
    "bsm_last_error": (ctypes.c_char_p, []),
    "bsm_ctx_set_profiling": (c_int, [c_void_p, c_int]),
    "bsm_ctx_set_rows_per_wave": (c_int, [c_void_p, c_int]),
    "bsm_ctx_set_product_variant": (c_int, [c_void_p, c_int]),
    "bsm_ctx_set_group_span": (c_int, [c_void_p, c_int]),
    "bsm_ctx_set_column_order": (c_int, [c_void_p, c_int]),
    "bsm_ctx_set_transposed_plans": (c_int, [c_void_p, c_int]),
    "bsm_ctx_product_stats": (c_int, [c_void_p, ctypes.POINTER(_ProductStat), c_int, ctypes.POINTER(c_int)]),
    "bsm_create_pattern": (c_int, [c_void_p, c_int, c_int, c_void_p, ctypes.POINTER(c_double), c_double,
                                   ctypes.POINTER(c_void_p)]),
    "bsm_pattern_destroy": (c_int, [c_void_p]),
    "bsm_pattern_get_info": (c_int, [c_void_p, ctypes.POINTER(_PatternInfo)]),
    "bsm_pattern_copy_to_host": (c_int, [c_void_p, c_void_p, c_void_p]),
    "bsm_matrix_fill_blocks": (c_int, [c_void_p, ctypes.POINTER(_Matrix), c_int64, c_void_p, c_void_p,
                                       c_void_p]),
    "bsm_axpby": (c_int, [c_void_p, c_double, ctypes.POINTER(_Matrix), c_double, ctypes.POINTER(_Matrix)]),
    "bsm_symmetrize": (c_int, [c_void_p, ctypes.POINTER(_Matrix)]),
    "bsm_mask_copy": (c_int, [c_void_p, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix)]),
    "bsm_set_identity": (c_int, [c_void_p, ctypes.POINTER(_Matrix), c_double]),
    "bsm_dot": (c_int, [c_void_p, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix), ctypes.POINTER(c_double)]),
    "bsm_multiply_truncate": (c_int, [c_void_p, c_double, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix),
                                      c_double, ctypes.POINTER(_Matrix)]),
    "bsm_multiply_truncate_pair": (c_int, [c_void_p, c_double, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix),
                                           ctypes.POINTER(_Matrix), c_double, ctypes.POINTER(_Matrix),
                                           ctypes.POINTER(_Matrix)]),
    "bsm_multiply_truncate_pair_a": (c_int, [c_void_p, c_double, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix),
                                             ctypes.POINTER(_Matrix), c_double, ctypes.POINTER(_Matrix),
                                             ctypes.POINTER(_Matrix)]),
    "bsm_product_flops": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double)]),
    "bsm_multiply_truncate_prec": (c_int, [c_void_p, c_int, c_double, ctypes.POINTER(_Matrix),
                                           ctypes.POINTER(_Matrix), c_double, ctypes.POINTER(_Matrix)]),
    "bsm_trace_product": (c_int, [c_void_p, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix),
                                  ctypes.POINTER(c_double)]),
    "bsm_trace_product_noalloc": (c_int, [c_void_p, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix), c_void_p]),
    "bsm_batch_create": (c_int, [c_void_p, c_int, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix),
                                 ctypes.POINTER(_Matrix), ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                 c_int, ctypes.POINTER(c_void_p)]),
    "bsm_batch_run": (c_int, [c_void_p, ctypes.POINTER(_BatchConfig)]),
    "bsm_batch_tune": (c_int, [c_void_p, c_int, ctypes.POINTER(_BatchConfig), ctypes.POINTER(c_double)]),
    "bsm_batch_flops": (c_int, [c_void_p, ctypes.POINTER(c_double)]),
    "bsm_batch_destroy": (c_int, [c_void_p]),
    "hotelling_inverse": (c_int, [c_void_p, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix),
                                  ctypes.POINTER(_HotParams), ctypes.POINTER(_HotResult)]),
    "bsm_contract": (c_int, [c_void_p, ctypes.POINTER(_Matrix), c_void_p, ctypes.POINTER(_Matrix)]),
    "bsm_inverse_sqrt": (c_int, [c_void_p, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix),
                                 ctypes.POINTER(_Matrix), ctypes.POINTER(_HotParams), ctypes.POINTER(_HotResult)]),
    "lnv_state_create": (c_int, [c_void_p, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix),
                                 ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix), ctypes.POINTER(_LNVParams),
                                 ctypes.POINTER(c_void_p)]),
    "lnv_step": (c_int, [c_void_p, ctypes.POINTER(_LNVResult)]),
    "lnv_state_destroy": (c_int, [c_void_p]),
    "lnv_state_reset": (c_int, [c_void_p, ctypes.POINTER(_LNVParams), ctypes.POINTER(c_double)]),
    "lnv_solve": (c_int, [c_void_p, ctypes.POINTER(_LNVSchedule), ctypes.POINTER(_LNVSolveResult)]),
    "lnv_idempotency_error": (c_int, [c_void_p, ctypes.POINTER(c_double)]),
    "lnv_forces": (c_int, [c_void_p, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix),
                           ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
    # learned initial guess (include/bsm_guess.h)
    "bsm_mlp_param_count": (c_int64, [ctypes.POINTER(_MlpShape)]),
    "bsm_mlp_create": (c_int, [c_void_p, ctypes.POINTER(_MlpShape), c_void_p, ctypes.POINTER(c_void_p)]),
    "bsm_mlp_get_params": (c_int, [c_void_p, c_void_p]),
    "bsm_mlp_set_params": (c_int, [c_void_p, c_void_p]),
    "bsm_mlp_destroy": (c_int, [c_void_p]),
    "bsm_pair_descriptors": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "bsm_mlp_forward": (c_int, [c_void_p, c_int, c_int64, c_void_p, c_void_p]),
    "bsm_mlp_loss_grad": (c_int, [c_void_p, c_int64, c_void_p, c_void_p, ctypes.POINTER(c_double), c_void_p]),
    "bsm_mlp_adam_step": (c_int, [c_void_p, ctypes.POINTER(_Adam), c_void_p]),
    "bsm_mlp_train": (c_int, [c_void_p, ctypes.POINTER(_TrainParams), c_int64, c_void_p, c_void_p, c_void_p,
                              ctypes.POINTER(c_double)]),
    "bsm_mlp_targets": (c_int, [c_void_p, ctypes.POINTER(_Matrix), ctypes.POINTER(_Matrix), c_double, c_void_p]),
    "bsm_mlp_predict_blocks": (c_int, [c_void_p, c_int, c_void_p, c_double, c_double, ctypes.POINTER(_Matrix)]),
    "lnv_state_reset_guess": (c_int, [c_void_p, ctypes.POINTER(_LNVParams), ctypes.POINTER(_Matrix), c_double,
                                      ctypes.POINTER(_GuessResult)]),
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2205_08941_amd/build.py` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = load_library()


def _check(code: int) -> None:
    if code != OK:
        raise BSMError(code, _lib.bsm_last_error().decode(errors="replace"))


# ---------------------------------------------------------------- objects
_LIVE_CONTEXTS = weakref.WeakSet()


def _close_all():
    for c in list(_LIVE_CONTEXTS):
        c.close()


atexit.register(_close_all)


class Context:
    """Library context on one GPU; all work goes to `stream` (default: torch's current).

    Patterns and LNV states created on a context are released before it, and
    everything is released at interpreter exit while Python is still alive.
    """

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 use_torch_allocator: bool = True):
        self._children = weakref.WeakSet()
        self.handle = None
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._keep = {}
        self._alloc_cb = ALLOC_FN(self._alloc) if use_torch_allocator else ALLOC_FN()
        self._free_cb = FREE_FN(self._free) if use_torch_allocator else FREE_FN()
        h = c_void_p()
        _check(_lib.bsm_ctx_create(device, c_void_p(self.stream.cuda_stream), self._alloc_cb,
                                   self._free_cb, None, ctypes.byref(h)))
        self.handle = h
        _LIVE_CONTEXTS.add(self)

    def set_profiling(self, enable: bool) -> None:
        """Time every product launch with HIP events on this context's stream."""
        _check(_lib.bsm_ctx_set_profiling(self.handle, int(bool(enable))))

    def set_rows_per_wave(self, rows: int) -> None:
        """Rows per wavefront tile (2, 4, 8; 0 = default) of plans built from now on."""
        _check(_lib.bsm_ctx_set_rows_per_wave(self.handle, int(rows)))

    def set_product_variant(self, variant: int) -> None:
        """Product kernel of plans built from now on: 0 SGPR A, 1 DPP-broadcast A, 2 workgroup
        tiles, 3 and 4 LDS-DMA rings (4: buffer copies), 5 rings with tiles shared by two
        waves, -1 the default (4 for b = 4 and 9).  Clears cached plans."""
        _check(_lib.bsm_ctx_set_product_variant(self.handle, int(variant)))

    def set_group_span(self, span: int) -> None:
        """Row groups interleaved by column position in the product launch order."""
        _check(_lib.bsm_ctx_set_group_span(self.handle, int(span)))

    def set_column_order(self, order: int) -> None:
        """Tile columns of plans built from now on: 0 ascending, 1 grouped by the rows they
        hold outputs for (default); same products either way.  Clears cached plans."""
        _check(_lib.bsm_ctx_set_column_order(self.handle, int(order)))

    def set_transposed_plans(self, mode: int) -> None:
        """Products of A and B on different patterns: 0 direct plans only, 1 (default) the
        cheaper of C = A B and C = (B^T A^T)^T, 2 the transposed plan whenever eligible.
        Results are equal either way.  Clears cached plans."""
        _check(_lib.bsm_ctx_set_transposed_plans(self.handle, int(mode)))

    def product_stats(self) -> list:
        """Per (P_A, P_B, P_C) class: launches, algorithmic flops, event milliseconds."""
        n = c_int()
        _check(_lib.bsm_ctx_product_stats(self.handle, None, 0, ctypes.byref(n)))
        arr = (_ProductStat * max(n.value, 1))()
        _check(_lib.bsm_ctx_product_stats(self.handle, arr, n.value, ctypes.byref(n)))
        return [dict(natoms=a.natoms, b=a.b, cutoffs=(a.cutoff_a, a.cutoff_b, a.cutoff_c),
                     launches=a.launches, flops=a.flops, ms=a.ms, variant=a.variant, rows=a.rows,
                     precision=a.precision, products=a.products) for a in arr[: n.value]]

    def _alloc(self, nbytes, user):
        try:
            with torch.cuda.stream(self.stream):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:
            return None
        p = t.data_ptr()
        self._keep[p] = t
        return p

    def _free(self, ptr, user):
        self._keep.pop(ptr, None)

    def close(self):
        # solver states and batches before the patterns they point into
        for ch in sorted(self._children, key=lambda o: not isinstance(o, (LNV, Batch, MLP))):
            ch.close()
        if self.handle:
            _lib.bsm_ctx_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        if not sys.is_finalizing():
            self.close()


class Pattern:
    """P_cutoff over the atoms at `positions` (built on the GPU)."""

    def __init__(self, ctx: Context, positions, box, cutoff: float, b: int):
        self.ctx = ctx
        pos = torch.as_tensor(np.asarray(positions, np.float64) if not torch.is_tensor(positions) else positions,
                              dtype=torch.float64).to(ctx.device).contiguous()
        bx = (c_double * 3)(*[float(v) for v in box])
        h = c_void_p()
        _check(_lib.bsm_create_pattern(ctx.handle, pos.shape[0], int(b), c_void_p(pos.data_ptr()), bx,
                                       float(cutoff), ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)
        info = _PatternInfo()
        _check(_lib.bsm_pattern_get_info(h, ctypes.byref(info)))
        self.natoms, self.b, self.nnzb, self.max_row = info.natoms, info.b, info.nnzb, info.max_row
        self.cutoff, self.box = info.cutoff, tuple(info.box)

    def to_host(self):
        rp = np.zeros(self.natoms + 1, np.int32)
        cols = np.zeros(max(self.nnzb, 1), np.int32)
        _check(_lib.bsm_pattern_copy_to_host(self.handle, rp.ctypes.data_as(c_void_p),
                                             cols.ctypes.data_as(c_void_p)))
        return rp, cols[: self.nnzb]

    def close(self):
        if getattr(self, "handle", None) and self.ctx.handle:
            _lib.bsm_pattern_destroy(self.handle)
        self.handle = None

    def __del__(self):
        if not sys.is_finalizing():
            self.close()


class Matrix:
    """Block-sparse FP64 matrix on a pattern: blocks is a device tensor (nnzb, b, b)."""

    def __init__(self, pattern: Pattern, blocks: Optional[torch.Tensor] = None):
        self.pattern = pattern
        shape = (pattern.nnzb, pattern.b, pattern.b)
        if blocks is None:
            blocks = torch.zeros(shape, dtype=torch.float64, device=pattern.ctx.device)
        assert blocks.dtype == torch.float64 and tuple(blocks.shape) == shape and blocks.is_contiguous()
        self.blocks = blocks
        self._c = _Matrix(pattern.handle, F64, c_void_p(blocks.data_ptr()))

    @property
    def c(self):
        return ctypes.byref(self._c)


def fill_blocks(M: Matrix, rows, cols, blocks) -> None:
    """M <- 0, then place the given blocks (must fall inside M's pattern)."""
    dev = M.pattern.ctx.device
    r = torch.as_tensor(np.asarray(rows, np.int32)).to(dev)
    c = torch.as_tensor(np.asarray(cols, np.int32)).to(dev)
    b = torch.as_tensor(np.ascontiguousarray(blocks, np.float64)).to(dev)
    _check(_lib.bsm_matrix_fill_blocks(M.pattern.ctx.handle, M.c, len(r), c_void_p(r.data_ptr()),
                                       c_void_p(c.data_ptr()), c_void_p(b.data_ptr())))


def multiply_truncate(alpha: float, A: Matrix, B: Matrix, beta: float, C: Matrix) -> None:
    _check(_lib.bsm_multiply_truncate(C.pattern.ctx.handle, float(alpha), A.c, B.c, float(beta), C.c))


def multiply_truncate_pair(alpha: float, A: Matrix, A2: Matrix, B: Matrix, beta: float, C: Matrix,
                           C2: Matrix) -> None:
    """C <- alpha mask(A B) + beta C and C2 <- alpha mask(A2 B) + beta C2 in one launch (A, A2 on one
    pattern, C, C2 on one pattern)."""
    _check(_lib.bsm_multiply_truncate_pair(C.pattern.ctx.handle, float(alpha), A.c, A2.c, B.c, float(beta), C.c,
                                           C2.c))


def multiply_truncate_pair_a(alpha: float, A: Matrix, B: Matrix, B2: Matrix, beta: float, C: Matrix,
                             C2: Matrix) -> None:
    """C <- alpha mask(A B) + beta C and C2 <- alpha mask(A B2) + beta C2 in one launch (B, B2 on one
    pattern, C, C2 on one pattern)."""
    _check(_lib.bsm_multiply_truncate_pair_a(C.pattern.ctx.handle, float(alpha), A.c, B.c, B2.c, float(beta), C.c,
                                             C2.c))


def multiply_truncate_prec(precision: int, alpha: float, A: Matrix, B: Matrix, beta: float, C: Matrix) -> None:
    """The product with inputs rounded to F32 or BF16 and FP32 accumulation (F64: exact)."""
    _check(_lib.bsm_multiply_truncate_prec(C.pattern.ctx.handle, int(precision), float(alpha), A.c, B.c,
                                           float(beta), C.c))


def product_flops(PA: Pattern, PB: Pattern, PC: Pattern) -> float:
    f = c_double()
    _check(_lib.bsm_product_flops(PC.ctx.handle, PA.handle, PB.handle, PC.handle, ctypes.byref(f)))
    return f.value


def trace_product(A: Matrix, B: Matrix) -> float:
    out = c_double()
    _check(_lib.bsm_trace_product(A.pattern.ctx.handle, A.c, B.c, ctypes.byref(out)))
    return out.value


def trace_product_noalloc(A: Matrix, B: Matrix, out: torch.Tensor) -> None:
    """Tr(A B) into out[0] (a float64 tensor on the device), asynchronously, with no
    allocation in the library (its partial sums sit in a static device array shared by
    every call on the GPU: overlapping calls race)."""
    if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 1:
        raise ValueError("out must be a float64 device tensor with at least one element")
    _check(_lib.bsm_trace_product_noalloc(A.pattern.ctx.handle, A.c, B.c, c_void_p(out.data_ptr())))


def dot(A: Matrix, B: Matrix) -> float:
    out = c_double()
    _check(_lib.bsm_dot(A.pattern.ctx.handle, A.c, B.c, ctypes.byref(out)))
    return out.value


def axpby(alpha: float, X: Matrix, beta: float, Y: Matrix) -> None:
    _check(_lib.bsm_axpby(Y.pattern.ctx.handle, float(alpha), X.c, float(beta), Y.c))


def symmetrize(M: Matrix) -> None:
    _check(_lib.bsm_symmetrize(M.pattern.ctx.handle, M.c))


def mask_copy(src: Matrix, dst: Matrix) -> None:
    _check(_lib.bsm_mask_copy(dst.pattern.ctx.handle, src.c, dst.c))


def set_identity(M: Matrix, alpha: float = 1.0) -> None:
    _check(_lib.bsm_set_identity(M.pattern.ctx.handle, M.c, float(alpha)))


class Batch:
    """Independent products C_p <- alpha_p mask(A_p B_p) + beta_p C_p in one persistent launch."""

    def __init__(self, ctx: Context, triples, alpha=1.0, beta=0.0, precision: int = F64):
        self.ctx = ctx
        self.triples = list(triples)          # keep the matrices alive
        n = len(self.triples)
        A = (_Matrix * n)(*[t[0]._c for t in self.triples])
        B = (_Matrix * n)(*[t[1]._c for t in self.triples])
        C = (_Matrix * n)(*[t[2]._c for t in self.triples])
        al = (c_double * n)(*([float(alpha)] * n if np.isscalar(alpha) else [float(a) for a in alpha]))
        be = (c_double * n)(*([float(beta)] * n if np.isscalar(beta) else [float(b) for b in beta]))
        h = c_void_p()
        _check(_lib.bsm_batch_create(ctx.handle, n, A, B, C, al, be, int(precision), ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)
        f = c_double()
        _check(_lib.bsm_batch_flops(h, ctypes.byref(f)))
        self.flops = f.value

    def run(self, order: Optional[int] = None, waves_per_cu: int = 8, queues: int = 1,
            mode: int = BATCH_ONE_LAUNCH) -> None:
        """order None: the tuned (or default) schedule; else the given one (mode BATCH_ONE_LAUNCH,
        BATCH_PER_B or BATCH_SEPARATE)."""
        if order is None:
            _check(_lib.bsm_batch_run(self.handle, None))
        else:
            cfg = _BatchConfig(int(order), int(waves_per_cu), int(queues), int(mode))
            _check(_lib.bsm_batch_run(self.handle, ctypes.byref(cfg)))

    def tune(self, reps: int = 1):
        cfg, ms = _BatchConfig(), c_double()
        _check(_lib.bsm_batch_tune(self.handle, int(reps), ctypes.byref(cfg), ctypes.byref(ms)))
        return dict(order=cfg.order, waves_per_cu=cfg.waves_per_cu, queues=cfg.queues, mode=cfg.mode), ms.value

    def close(self):
        if getattr(self, "handle", None) and self.ctx.handle:
            _lib.bsm_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        if not sys.is_finalizing():
            self.close()


@dataclass
class HotellingResult:
    status: int
    iterations: int
    alpha: float
    residuals: List[float]
    product_flops: float = 0.0
    start: int = 0


INIT_PLAIN, INIT_GIVEN, INIT_GUARDED = 0, 1, 2


def hotelling_inverse(S: Matrix, Z: Matrix, max_iter: int = 100, tol: float = 1e-12,
                      init_given: int = INIT_PLAIN, raise_on_error: bool = True) -> HotellingResult:
    """init_given: INIT_PLAIN (I / rho), INIT_GIVEN (Z's contents) or INIT_GUARDED (Z's contents
    when they start closer to S^-1, with I / rho as fallback); True / False mean GIVEN / PLAIN."""
    cap = 2 * max_iter + 4
    buf = (c_double * cap)()
    prm = _HotParams(int(max_iter), float(tol), int(init_given))
    res = _HotResult(0, 0, 0.0, ctypes.cast(buf, ctypes.POINTER(c_double)), cap, 0, 0.0, 0)
    code = _lib.hotelling_inverse(Z.pattern.ctx.handle, S.c, Z.c, ctypes.byref(prm), ctypes.byref(res))
    if code != OK and raise_on_error:
        _check(code)
    return HotellingResult(res.status, res.iterations, res.alpha, list(buf[: min(res.n_residuals, cap)]),
                           res.product_flops, res.start)


def contract(M: Matrix, coef: torch.Tensor, out: Matrix) -> None:
    """out <- blocks C_i^T M_ij C_j; coef a device float64 tensor (natoms, b, bc), bc = out's b."""
    assert coef.dtype == torch.float64 and coef.is_cuda and coef.is_contiguous()
    assert tuple(coef.shape) == (M.pattern.natoms, M.pattern.b, out.pattern.b)
    _check(_lib.bsm_contract(out.pattern.ctx.handle, M.c, c_void_p(coef.data_ptr()), out.c))


def inverse_sqrt(S: Matrix, Z: Matrix, Y: Optional[Matrix] = None, max_iter: int = 100, tol: float = 1e-12,
                 raise_on_error: bool = True) -> HotellingResult:
    """S^-1/2 into Z (and S^1/2 into Y, on Z's pattern, when given) by the truncated
    coupled Newton-Schulz iteration; result fields as for hotelling_inverse."""
    cap = max_iter + 4
    buf = (c_double * cap)()
    prm = _HotParams(int(max_iter), float(tol), INIT_PLAIN)
    res = _HotResult(0, 0, 0.0, ctypes.cast(buf, ctypes.POINTER(c_double)), cap, 0, 0.0, 0)
    code = _lib.bsm_inverse_sqrt(Z.pattern.ctx.handle, S.c, Z.c, Y.c if Y is not None else None,
                                 ctypes.byref(prm), ctypes.byref(res))
    if code != OK and raise_on_error:
        _check(code)
    return HotellingResult(res.status, res.iterations, res.alpha, list(buf[: min(res.n_residuals, cap)]),
                           res.product_flops, res.start)


@dataclass
class LNVResult:
    E: float
    Omega: float
    N: float
    mu: float
    alpha: float
    beta: float
    dE: float
    c: tuple
    converged: bool
    status: int
    product_flops: float


class LNV:
    """LNV minimisation state over L's pattern; L (a Matrix) is updated in place."""

    def __init__(self, S: Matrix, H: Matrix, Z: Matrix, L: Matrix, n_electrons: float, mode: int = CANONICAL,
                 mu: float = 0.0, tol_E: float = 1e-8, init_from_z: bool = True, precision: int = F64):
        self.ctx = L.pattern.ctx
        self.S, self.H, self.Z, self.L = S, H, Z, L   # keep the device buffers alive
        self.n_electrons, self.mode, self.mu, self.tol_E = float(n_electrons), int(mode), float(mu), float(tol_E)
        self.precision = int(precision)
        prm = _LNVParams(float(n_electrons), int(mode), float(mu), float(tol_E), int(bool(init_from_z)),
                         self.precision)
        h = c_void_p()
        _check(_lib.lnv_state_create(self.ctx.handle, S.c, H.c, Z.c, L.c, ctypes.byref(prm), ctypes.byref(h)))
        self.handle = h
        self.ctx._children.add(self)

    def reset(self, init_from_z: bool = True, precision: Optional[int] = None) -> float:
        """Restart from c mask_L(Z) (or the current L); returns the init products' flops."""
        if precision is not None:
            self.precision = int(precision)
        prm = _LNVParams(self.n_electrons, self.mode, self.mu, self.tol_E, int(bool(init_from_z)), self.precision)
        f = c_double()
        _check(_lib.lnv_state_reset(self.handle, ctypes.byref(prm), ctypes.byref(f)))
        return f.value

    def step(self, raise_on_error: bool = False) -> LNVResult:
        r = _LNVResult()
        code = _lib.lnv_step(self.handle, ctypes.byref(r))
        if code != OK and raise_on_error:
            _check(code)
        return LNVResult(r.E, r.Omega, r.N, r.mu, r.alpha, r.beta, r.dE, tuple(r.c), bool(r.converged),
                         r.status, r.product_flops)

    def reset_guess(self, dL: Matrix, n_tol: float = 0.01, precision: Optional[int] = None) -> dict:
        """Restart from c mask_L(Z) + dL when that start is better (lower E, N within n_tol N_e),
        else from c mask_L(Z)."""
        if precision is not None:
            self.precision = int(precision)
        prm = _LNVParams(self.n_electrons, self.mode, self.mu, self.tol_E, 1, self.precision)
        r = _GuessResult()
        _check(_lib.lnv_state_reset_guess(self.handle, ctypes.byref(prm), dL.c, float(n_tol), ctypes.byref(r)))
        return dict(accepted=bool(r.accepted), E_plain=r.E_plain, N_plain=r.N_plain, E_guess=r.E_guess,
                    N_guess=r.N_guess, product_flops=r.product_flops)

    def idempotency_error(self) -> float:
        """||mask(KS KS) - KS||_F / ||KS||_F of the current L (FP64)."""
        e = c_double()
        _check(_lib.lnv_idempotency_error(self.handle, ctypes.byref(e)))
        return e.value

    def forces(self, dS: Sequence[Matrix], dH: Sequence[Matrix]):
        """(forces (natoms, 3) as numpy, mu) at the current L; dS, dH: the x, y, z derivative
        matrices on S's and H's patterns (d block_ij / d R_j)."""
        assert len(dS) == 3 and len(dH) == 3
        ms = (_Matrix * 3)(*[m._c for m in dS])
        mh = (_Matrix * 3)(*[m._c for m in dH])
        n = self.S.pattern.natoms
        out = (c_double * (3 * n))()
        mu = c_double()
        _check(_lib.lnv_forces(self.handle, ms, mh, out, ctypes.byref(mu)))
        return np.frombuffer(out, dtype=np.float64).reshape(n, 3).copy(), mu.value

    def solve(self, stages) -> dict:
        """Run a precision schedule: stages = [(precision, max_iter, tol_E, stop_on_rise), ...]."""
        sch = _LNVSchedule()
        sch.n_stages = len(stages)
        for k, (p, mi, tol, rise) in enumerate(stages):
            sch.precision[k], sch.max_iter[k], sch.tol_E[k], sch.stop_on_rise[k] = int(p), int(mi), float(tol), int(rise)
        r = _LNVSolveResult()
        code = _lib.lnv_solve(self.handle, ctypes.byref(sch), ctypes.byref(r))
        return dict(status=code, converged=bool(r.converged), iterations=list(r.iterations)[: len(stages)],
                    E=r.E, N=r.N, mu=r.mu, product_flops=r.product_flops)

    def close(self):
        if getattr(self, "handle", None) and self.ctx.handle:
            _lib.lnv_state_destroy(self.handle)
        self.handle = None

    def __del__(self):
        if not sys.is_finalizing():
            self.close()


# --------------------------------------------------------------------------- learned initial guess

DESC_DIM, MLP_WIDTH = 32, 128


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else c_void_p(t.data_ptr())


def pair_descriptors(neighbours: Pattern, P: Pattern) -> torch.Tensor:
    """(nnzb(P), 16) FP32 descriptors of P's slots; frames from the four nearest atoms in `neighbours`."""
    X = torch.empty((max(P.nnzb, 1), DESC_DIM), dtype=torch.float32, device=P.ctx.device)
    _check(_lib.bsm_pair_descriptors(P.ctx.handle, neighbours.handle, P.handle, _ptr(X)))
    return X[: P.nnzb]


def mlp_targets(A: Matrix, B: Matrix, scale: float) -> torch.Tensor:
    """(nnzb, b^2) FP32 training targets (A - B) / scale."""
    P = A.pattern
    T = torch.empty((max(P.nnzb, 1), P.b * P.b), dtype=torch.float32, device=P.ctx.device)
    _check(_lib.bsm_mlp_targets(P.ctx.handle, A.c, B.c, float(scale), _ptr(T)))
    return T[: P.nnzb]


def mlp_param_count(out_dim: int, width: int = MLP_WIDTH) -> int:
    n = _lib.bsm_mlp_param_count(ctypes.byref(_MlpShape(int(width), int(out_dim))))
    if n < 0:
        _check(int(n))
    return int(n)


class MLP:
    """Three-layer perceptron on the GPU (parameters FP32; the caller supplies the initial values)."""

    def __init__(self, ctx: Context, out_dim: int, params, width: int = MLP_WIDTH):
        self.ctx, self.out_dim, self.width = ctx, int(out_dim), int(width)
        self.count = mlp_param_count(out_dim, width)
        p = np.ascontiguousarray(params, np.float32)
        assert p.shape == (self.count,), (p.shape, self.count)
        h = c_void_p()
        _check(_lib.bsm_mlp_create(ctx.handle, ctypes.byref(_MlpShape(self.width, self.out_dim)),
                                   p.ctypes.data_as(c_void_p), ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)

    @property
    def params(self) -> np.ndarray:
        p = np.empty(self.count, np.float32)
        _check(_lib.bsm_mlp_get_params(self.handle, p.ctypes.data_as(c_void_p)))
        return p

    @params.setter
    def params(self, values) -> None:
        p = np.ascontiguousarray(values, np.float32)
        assert p.shape == (self.count,)
        _check(_lib.bsm_mlp_set_params(self.handle, p.ctypes.data_as(c_void_p)))

    def forward(self, X: torch.Tensor, precision: int = F32) -> torch.Tensor:
        X = X.contiguous()
        Y = torch.empty((max(X.shape[0], 1), self.out_dim), dtype=torch.float32, device=X.device)
        _check(_lib.bsm_mlp_forward(self.handle, int(precision), X.shape[0], _ptr(X), _ptr(Y)))
        return Y[: X.shape[0]]

    def loss_grad(self, X: torch.Tensor, T: torch.Tensor):
        g = torch.empty(self.count, dtype=torch.float32, device=X.device)
        loss = c_double()
        _check(_lib.bsm_mlp_loss_grad(self.handle, X.shape[0], _ptr(X.contiguous()), _ptr(T.contiguous()),
                                      ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def adam_step(self, grad: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
        _check(_lib.bsm_mlp_adam_step(self.handle, ctypes.byref(_Adam(lr, beta1, beta2, eps)), _ptr(grad)))

    def train(self, X: torch.Tensor, T: torch.Tensor, epochs: int, batch: int, lr=1e-3, beta1=0.9,
              beta2=0.999, eps=1e-8, perm: Optional[torch.Tensor] = None) -> List[float]:
        """Minibatch Adam; perm (int32 device tensor) orders the samples.  Returns per-epoch mean losses."""
        losses = (c_double * max(int(epochs), 1))()
        prm = _TrainParams(int(epochs), int(batch), _Adam(lr, beta1, beta2, eps))
        if perm is not None:
            assert perm.dtype == torch.int32 and perm.numel() == X.shape[0]
        _check(_lib.bsm_mlp_train(self.handle, ctypes.byref(prm), X.shape[0], _ptr(X.contiguous()),
                                  _ptr(T.contiguous()), _ptr(perm), losses))
        return list(losses[: int(epochs)])

    def predict_blocks(self, X: torch.Tensor, M: Matrix, scale: float = 1.0, beta: float = 0.0,
                       precision: int = F32) -> None:
        """M <- beta M + scale * network(X), X the descriptors of M's pattern."""
        _check(_lib.bsm_mlp_predict_blocks(self.handle, int(precision), _ptr(X.contiguous()), float(scale),
                                           float(beta), M.c))

    def close(self):
        if getattr(self, "handle", None) and self.ctx.handle:
            _lib.bsm_mlp_destroy(self.handle)
        self.handle = None

    def __del__(self):
        if not sys.is_finalizing():
            self.close()
