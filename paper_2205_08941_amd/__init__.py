"""MI355X (gfx950) block-sparse linear-scaling DFT hot path: truncated block
products, traces, Hotelling S^-1, Newton-Schulz S^-1/2 and LNV minimisation in hand-written HIP,
behind the C ABI of include/bsm.h, and the learned initial guess of
include/bsm_guess.h.  Importing this package loads libbsm.so
and fails if it has not been built; there is no CPU fallback."""
from .bsm import (BSMError, Context, Pattern, Matrix, LNV, Batch, ORDER_BY_PRODUCT, ORDER_HEAVY_FIRST,
                  ORDER_INTERLEAVE, BATCH_ONE_LAUNCH, BATCH_PER_B, BATCH_SEPARATE, LNVResult, HotellingResult, fill_blocks,
                  multiply_truncate, multiply_truncate_pair, multiply_truncate_pair_a, multiply_truncate_prec, product_flops, trace_product, trace_product_noalloc, dot, axpby, symmetrize, mask_copy,
                  set_identity, hotelling_inverse, inverse_sqrt, contract, load_library, LIB_PATH, EXPORTS,
                  OK, EINVAL, ENOMEM, EPATTERN, EHIP, ENONFINITE, EDIVERGED, ENOTCONV, ERUNAWAY,
                  CANONICAL, GRAND, F64, F32, BF16,
                  MLP, pair_descriptors, mlp_targets, mlp_param_count, DESC_DIM, MLP_WIDTH,
                  INIT_PLAIN, INIT_GIVEN, INIT_GUARDED)
