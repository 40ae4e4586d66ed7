/*
 * bsm.h -- C ABI of the MI355X (gfx950) block-sparse linear-scaling DFT hot path.
 *
 * The paper (Bowler, Miyazaki, Nakata, Truflandier, "The CONQUEST code: large
 * scale and linear scaling DFT") describes a ground-state solver built on
 * sparse matrix storage and operations that keep every step local (section
 * "Background and Current Status"), whose linear-scaling form depends on
 * inverting the overlap matrix in linear time (section "Development
 * Priorities"), and which it plans to run entirely on GPUs (section "Meeting
 * the Exascale Challenges").  This library is that GPU solver's data-parallel
 * core: atom-block sparse matrices truncated to spatial-cutoff patterns, their
 * products and traces, the Hotelling iteration for S^-1 and the LNV
 * (Li-Nunes-Vanderbilt) density-matrix minimisation with K = 3LSL - 2LSLSL.
 *
 * Conventions (all entry points):
 *   - Return BSM_OK (0) on success and a negative BSM_E* code on failure;
 *     bsm_last_error() then gives a message (thread-local, valid until the next
 *     failing call on the same thread).  No C++ exception crosses this ABI.
 *   - "device" pointers are HIP device memory of the context's device; "host"
 *     pointers are ordinary CPU memory.
 *   - Work is queued on the context's stream.  Calls that return a host scalar
 *     (traces, dots, drivers) synchronise that stream; the others are
 *     asynchronous.
 *   - A failed call leaves its outputs unspecified and every handle valid.
 *   - A context and everything created from it must be used from one host
 *     thread at a time.
 *
 * Storage:
 *   - A pattern P_r over N atoms holds every ordered atom pair (i, j) whose
 *     minimum-image distance in the orthorhombic periodic box is strictly below
 *     r (compared as d^2 < r^2 in FP64, no fused multiply-add), plus (i, i).
 *     It is block CSR: row i lists its columns j in ascending order.  Patterns
 *     are symmetric by construction.
 *   - A matrix on a pattern with b orbitals per atom stores one b x b block per
 *     pattern entry, row-major inside the block, blocks in CSR order:
 *     nnzb * b * b elements.  Blocks are Gamma-point folded (the block of (i, j)
 *     sums every periodic image of the pair).
 *   - Atom order is the caller's; the library never permutes atoms.  Spatially
 *     sorted atoms (Morton order) give better cache reuse in the products.
 */
#ifndef BSM_H
#define BSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BSM_OK = 0,
    BSM_EINVAL = -1,      /* bad argument (sizes, null pointers, aliasing) */
    BSM_ENOMEM = -2,      /* device allocation failed */
    BSM_EPATTERN = -3,    /* patterns or orbital counts do not match */
    BSM_EHIP = -4,        /* a HIP runtime call failed */
    BSM_ENONFINITE = -5,  /* a trace, residual or energy is NaN or infinite */
    BSM_EDIVERGED = -6,   /* Hotelling residual grew: S not positive definite */
    BSM_ENOTCONV = -7,    /* iteration limit reached before the tolerance */
    BSM_ERUNAWAY = -8     /* LNV line search found no minimum (outside the basin) */
};

enum { BSM_F64 = 0, BSM_F32 = 1, BSM_BF16 = 2 };

typedef struct bsm_ctx_s *bsm_ctx;
typedef struct bsm_pattern_s *bsm_pattern;

/* Optional allocator for all memory the library allocates itself (patterns,
 * plans, driver scratch).  Must return device memory of the context's device,
 * 256-byte aligned, or NULL on failure.  NULL callbacks select hipMalloc/hipFree. */
typedef void *(*bsm_alloc_fn)(size_t bytes, void *user);
typedef void (*bsm_free_fn)(void *ptr, void *user);

/* A matrix view.  `blocks` is caller-owned device memory of
 * nnzb(pattern) * b * b elements of `dtype`; the library never frees it. */
typedef struct {
    bsm_pattern pattern;
    int dtype;            /* BSM_F64 for every entry point of this header */
    void *blocks;
} bsm_matrix;

typedef struct {
    int natoms;
    int b;                /* orbitals per atom */
    int64_t nnzb;         /* number of blocks */
    int max_row;          /* longest row, in blocks */
    double cutoff;        /* Angstrom */
    double box[3];        /* Angstrom */
    const int32_t *rowptr;  /* device, natoms + 1 */
    const int32_t *cols;    /* device, nnzb, ascending within a row */
    const int32_t *tmap;    /* device, nnzb: slot of (j, i) for slot (i, j) */
    const int32_t *diag;    /* device, natoms: slot of (i, i) */
    const double *pos;      /* device, natoms * 3: the positions it was built from */
} bsm_pattern_info;

/* ---- context --------------------------------------------------------- */

/* Create a context on HIP device `device` queueing work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  The context owns plan caches and
 * reduction scratch.  Errors: BSM_EINVAL (out NULL or bad device), BSM_EHIP. */
int bsm_ctx_create(int device, void *hip_stream, bsm_alloc_fn alloc, bsm_free_fn free_fn,
                   void *user, bsm_ctx *out);
int bsm_ctx_destroy(bsm_ctx ctx);
int bsm_ctx_set_stream(bsm_ctx ctx, void *hip_stream);
const char *bsm_last_error(void);

/* Per-class timing of block products: with profiling on, every product launch
 * (from any entry point, drivers included) is bracketed by HIP events on the
 * context's stream.  Classes are (P_A, P_B, P_C) triples with the kernel
 * variant, rows per tile and operand precision of the launches. */
typedef struct {
    int natoms, b;
    double cutoff_a, cutoff_b, cutoff_c;  /* Angstrom */
    int64_t launches;
    double flops;        /* algorithmic flops summed over the launches */
    double ms;           /* summed event time, milliseconds */
    int variant, rows;   /* kernel variant (bsm_ctx_set_product_variant) and rows per tile */
    int precision;       /* BSM_F64, BSM_F32 or BSM_BF16 */
    int products;        /* products per launch: 1, or 2 for the paired launches */
} bsm_product_stat;

/* Rows of C per wavefront tile in product plans built from now on: 2, 4 or 8
 * (0 restores the default: 8 for the default kernel with b = 4 and 9, else 4
 * for b >= 4 and 2 below); variant 2 plans always use
 * 16-row workgroup tiles.  Larger values reuse each B block across more rows at
 * the cost of idle lanes.  Clears cached plans (destroy batches first). */
int bsm_ctx_set_rows_per_wave(bsm_ctx ctx, int rows);
/* FP64 product kernel of plans built from now on: 0 = the uniform A block read
 * through the scalar cache into SGPRs; 1 = A held in VGPRs and broadcast by DPP
 * (b = 4 and 9, rows per wave 2 or 4; other shapes use 0); 2 = workgroup tiles
 * of 16 rows (4 wavefronts of 4 rows sharing the tile's B blocks, staged in
 * LDS, A as in 1; b = 4 and 9, else 0); 3 and 4 = the wave tiles of 1 with
 * both operands copied into a per-wave LDS ring by asynchronous LDS-DMA loads,
 * 2 (3, at 2 or 4 rows) or 1 (4, and 3 at 8 rows) entries ahead (b = 4 and 9,
 * rows 2, 4 or 8, else 0); 3 addresses the copies with 64-bit pointers, 4
 * through buffer resources when A and B each hold at most 0xfffff000 bytes
 * (else as 3); 5 = the rings of 4 with each tile of twice the columns shared by
 * the two waves of a workgroup: one list of k per tile, a half entry per wave
 * (A slots of the rows with outputs in that wave's columns, its B slots), a
 * barrier per entry so that both waves copy the same A blocks together (the
 * second copy is served from cache); rows 4 or 8 (2 gives 4); BF16 products at
 * b = 9 use one-wave plans on the matrix cores; 6 = the one-wave tiles of 4 with
 * FP64 products on the matrix cores (v_mfma_f64_16x16x4_f64, b = 9 only, other b
 * take 4; rows 4 or 8; direct plans; FP32 and BF16 products take 4), a measured
 * alternative that multiplies every block pair of its 16 x 16 tiles; -1 = default
 * (4 for b = 4 and 9, with 8 rows per tile, else 0).
 * Variants 1 to 4 multiply absent (k, j) blocks by zero instead of skipping
 * them, so a non-finite block of A can make other blocks of its output row
 * non-finite.  Clears cached plans (a bsm_batch made before keeps pointers to
 * them: destroy batches first). */
int bsm_ctx_set_product_variant(bsm_ctx ctx, int variant);
/* Launch order of product tiles in plans built from now on: tiles of `span`
 * consecutive row groups are interleaved by column position (1 = group by
 * group), so that groups over similar columns share B blocks in L2.
 * 1 <= span <= 4096 (default 4).  Clears cached plans. */
int bsm_ctx_set_group_span(bsm_ctx ctx, int span);

/* Columns of the tiles of product plans built from now on.  Each group of
 * rows-per-tile consecutive rows covers the union of its rows of P_C in tiles of
 * 64 / b columns: order 0 takes the union in ascending column order; order 1
 * (default) first groups the columns by the set of the group's rows that hold an
 * output in them, so that within a tile every row multiplies only where it has
 * outputs (fewer idle lanes, fewer copied A blocks, somewhat more entries).  For
 * finite operands FP64 and FP32 products are equal under both orders (each
 * element sums the same nonzero terms in ascending k); BF16 matrix-core products
 * pair entries differently and may differ in rounding.  order must be 0 or 1.  Clears cached plans (destroy batches first). */
int bsm_ctx_set_column_order(bsm_ctx ctx, int order);

/* Transposed plans for the default product kernel (variant 4, 4 or 8 rows per
 * tile, b = 4 or 9) when A and B lie on different patterns: the product is also
 * planned as C = (B^T A^T)^T, i.e. D = B^T A^T on P_C with blocks read transposed
 * and D's blocks stored transposed at the slots of (j, i) (patterns are
 * symmetric).  A wide A times a narrow B then walks the narrow pattern, leaving
 * fewer lanes idle.  mode 0: never; 1 (default): both plans are built once and
 * the one with the smaller estimated cost (rows multiplied + 4.5 x entries) is
 * kept; 2: always when eligible.  Each element sums the same terms in the same order either way, so
 * results are equal.  BF16 products on the matrix cores always use direct plans.
 * Clears cached plans (destroy batches first). */
int bsm_ctx_set_transposed_plans(bsm_ctx ctx, int mode);

/* enable != 0 clears the statistics and starts recording; 0 stops. */
int bsm_ctx_set_profiling(bsm_ctx ctx, int enable);
/* Synchronises the stream, then writes up to `max` classes (most time first)
 * and their total number to *count. */
int bsm_ctx_product_stats(bsm_ctx ctx, bsm_product_stat *out, int max, int *count);

/* ---- patterns (paper: sparse storage exploiting locality, Background) -- */

/* Build P_cutoff over `natoms` atoms at device positions `pos` (natoms x 3 FP64,
 * Angstrom) in the orthorhombic periodic box `box` (host, 3 FP64), with `b`
 * orbitals per atom.  GPU cell-list search (cells no smaller than the cutoff;
 * fewer than three cells along an axis falls back to scanning that whole axis).
 * The positions are copied.  Errors: BSM_EINVAL (natoms <= 0, b not in 1..16,
 * cutoff <= 0, box <= 0, a row longer than 8192 blocks), BSM_ENOMEM, BSM_EHIP. */
int bsm_create_pattern(bsm_ctx ctx, int natoms, int b, const double *pos, const double box[3],
                       double cutoff, bsm_pattern *out);
int bsm_pattern_destroy(bsm_pattern p);
int bsm_pattern_get_info(bsm_pattern p, bsm_pattern_info *out);
/* Copy rowptr (natoms + 1) and cols (nnzb) to host buffers; synchronises. */
int bsm_pattern_copy_to_host(bsm_pattern p, int32_t *rowptr_host, int32_t *cols_host);

/* ---- matrices: input and pattern-local operations ----------------------- */

/* M <- 0, then M[(rows[n], cols[n])] = blocks[n] for n < count.  rows, cols
 * (int32) and blocks (count * b * b FP64) are device arrays; (row, col) pairs
 * must be distinct.  Errors: BSM_EPATTERN if a block falls outside M's pattern
 * (synchronises to check), BSM_EINVAL. */
int bsm_matrix_fill_blocks(bsm_ctx ctx, const bsm_matrix *M, int64_t count, const int32_t *rows,
                           const int32_t *cols, const double *blocks);
/* Y <- alpha X + beta Y (same pattern; beta == 0 ignores Y's old contents). */
int bsm_axpby(bsm_ctx ctx, double alpha, const bsm_matrix *X, double beta, const bsm_matrix *Y);
/* M <- (M + M^T) / 2 blockwise, in place. */
int bsm_symmetrize(bsm_ctx ctx, const bsm_matrix *M);
/* dst <- mask_{P_dst}(src): blocks of src inside dst's pattern, zero elsewhere.
 * Same natoms and b.  Errors: BSM_EPATTERN, BSM_EINVAL (src aliases dst). */
int bsm_mask_copy(bsm_ctx ctx, const bsm_matrix *src, const bsm_matrix *dst);
/* M <- alpha I on M's pattern. */
int bsm_set_identity(bsm_ctx ctx, const bsm_matrix *M, double alpha);
/* *out = <A, B> = sum of elementwise products (same pattern); FP64; synchronises. */
int bsm_dot(bsm_ctx ctx, const bsm_matrix *A, const bsm_matrix *B, double *out);

/* ---- the hot path ------------------------------------------------------- */

/* C <- alpha mask_{P_C}(A B) + beta C.
 * Block (i, j) of C in P_C receives sum over k with (i,k) in P_A and (k,j) in
 * P_B of A_ik B_kj; pairs outside P_C are never formed (the truncation of a
 * product back to its cutoff pattern, the paper's local sparse operations,
 * Background).  beta == 0 ignores C's old contents.  The product plan for
 * (P_A, P_B, P_C) is built on first use and cached in the context (tiles of
 * rows x columns of C with their lists of k; see bsm_ctx_set_column_order and
 * bsm_ctx_set_transposed_plans).  With beta != 0 each element is
 * alpha s + beta c, each product and the sum rounded separately.
 * Asynchronous.  Errors: BSM_EPATTERN (natoms or b differ), BSM_EINVAL (C's
 * blocks alias A's or B's, dtype not F64), BSM_ENOMEM, BSM_EHIP. */
int bsm_multiply_truncate(bsm_ctx ctx, double alpha, const bsm_matrix *A, const bsm_matrix *B,
                          double beta, const bsm_matrix *C);

/* Two truncated products that share their right operand, in one launch:
 * C <- alpha mask_{P_C}(A B) + beta C and C2 <- alpha mask_{P_C}(A2 B) + beta C2,
 * with A and A2 on one pattern and C and C2 on one pattern (the same products as
 * bsm_multiply_truncate, Background).  For b = 4 and 9 with the default kernel,
 * while the pair's 4-row plan fits (free device memory of twice its estimated
 * size and a quarter of the device; it is cached beside the class's default
 * plan), the pair runs as tiles of twice the rows of that plan: every copied block
 * of B serves both products, and each element of C and C2 equals, bit for bit,
 * what bsm_multiply_truncate gives; otherwise the two products run one after the
 * other.  LNV evaluates W = X X and U = Y X this way.  Asynchronous.  Errors: as
 * bsm_multiply_truncate, and BSM_EPATTERN when A2 or C2 is not on A's or C's
 * pattern; BSM_EINVAL when C or C2 aliases an operand or each other. */
int bsm_multiply_truncate_pair(bsm_ctx ctx, double alpha, const bsm_matrix *A, const bsm_matrix *A2,
                               const bsm_matrix *B, double beta, const bsm_matrix *C, const bsm_matrix *C2);

/* Two truncated products that share their left operand, in one launch:
 * C <- alpha mask_{P_C}(A B) + beta C and C2 <- alpha mask_{P_C}(A B2) + beta C2,
 * with B and B2 on one pattern and C and C2 on one pattern (Background).  For
 * b = 4 and 9 with the default kernel, while its plan fits as above, the pair
 * runs on a transposed plan (C = (B^T A^T)^T, all patterns being symmetric; whatever
 * bsm_ctx_set_transposed_plans sets for single products) as tiles of twice the rows of
 * one 4-row plan, every copied block of A serving both products, each element
 * equal bit for bit to what bsm_multiply_truncate gives; otherwise the two
 * products run one after the other.  LNV evaluates X = L S with Y = L H, and
 * X_D = D S with Y_D = D H, this way.  Asynchronous.  Errors: as
 * bsm_multiply_truncate_pair, with B2 in the place of A2. */
int bsm_multiply_truncate_pair_a(bsm_ctx ctx, double alpha, const bsm_matrix *A, const bsm_matrix *B,
                                 const bsm_matrix *B2, double beta, const bsm_matrix *C, const bsm_matrix *C2);
/* The same product with every element of A and B first rounded to `precision`:
 * BSM_F32 (round to nearest even) or BSM_BF16 (to FP32, then to 8 significant
 * bits, nearest even); products accumulated in FP32 by fused multiply-adds over
 * k ascending, then the block's inner index ascending; the FP32 sum is widened
 * exactly to FP64 and C <- alpha sum + beta C in FP64.  Exception: BSM_BF16 with
 * b = 9, A and B on one pattern, kernel variant 3 or 4 and 4 or 8 rows per tile
 * runs on the matrix cores (products exact in FP32, summed in FP32 in the matrix
 * core's order), so its sums differ from the FMA chain by FP32 rounding.  BSM_F64 is bsm_multiply_truncate.  A and B stay FP64
 * in memory; their rounded (or packed) copies live in context scratch.  Used for
 * the low-precision stages of an LNV solve with FP64 traces and refinement (an
 * extension built on the method, not in the paper). */
int bsm_multiply_truncate_prec(bsm_ctx ctx, int precision, double alpha, const bsm_matrix *A,
                               const bsm_matrix *B, double beta, const bsm_matrix *C);
/* Contraction to support functions (the on-site equivalent of multi-site
 * support functions, Development Priorities): every block of M (b x b) becomes
 * M'_ij = C_i^T M_ij C_j (bc x bc) in out, whose pattern has the same atoms and
 * cutoff with bc = out's orbitals per atom (bc <= b).  coef: device,
 * natoms x b x bc doubles, C_i[a][alpha] at coef[(i b + a) bc + alpha], caller-owned.
 * Asynchronous on the context stream.  Errors: BSM_EPATTERN (patterns differ),
 * BSM_EINVAL (bc > b, aliasing). */
int bsm_contract(bsm_ctx ctx, const bsm_matrix *M, const double *coef, const bsm_matrix *out);
/* ---- many products in one persistent launch (an extension: uneven systems) 
 * A batch of independent products C_p <- alpha_p mask(A_p B_p) + beta_p C_p,
 * b = 4 or 9 (e.g. one per system of a batch of uneven systems), runs as one
 * launch of resident wavefronts that take tiles from work queues until the list
 * is exhausted.  Tiles are the 8-row LDS-ring tiles of the separate launches;
 * results equal the separate products bit for bit (tiles write disjoint
 * outputs), except BF16 with b = 9, which the batch multiplies on the VALU (FP32
 * fused multiply-adds, as the separate product with explicit rows per tile)
 * while the default separate product uses the matrix cores.  The schedule (bsm_batch_config) is chosen by
 * bsm_batch_tune, which times every candidate on the batch itself. */
typedef struct bsm_batch_s *bsm_batch;
enum { BSM_ORDER_BY_PRODUCT = 0, BSM_ORDER_HEAVY_FIRST = 1, BSM_ORDER_INTERLEAVE = 2 };
enum { BSM_BATCH_ONE_LAUNCH = 0, BSM_BATCH_PER_B = 1, BSM_BATCH_SEPARATE = 2 };
typedef struct {
    int order;          /* BSM_ORDER_*: work-list order */
    int waves_per_cu;   /* resident wavefronts per CU: 4, 8, ..., 32 */
    int queues;         /* 1 (one global queue) or 8 (one per XCD, equal-weight slices) */
    int mode;           /* BSM_BATCH_ONE_LAUNCH: one persistent launch over every product's tiles;
                           BSM_BATCH_PER_B: one persistent launch per orbital count, each kernel
                           compiled for that tile alone; BSM_BATCH_SEPARATE: each product in its own
                           launch, as bsm_multiply_truncate_prec runs it (order, waves and queues
                           unused) */
} bsm_batch_config;
/* n products; A, B, C arrays of n matrices (C_p must not overlap A_p or B_p),
 * alpha, beta arrays of n.  precision: BSM_F64, BSM_F32 or BSM_BF16 (as in
 * bsm_multiply_truncate_prec).  Builds (or reuses) each product's plan.  The
 * matrices must outlive the batch.  Errors: BSM_EINVAL (b not 4 or 9),
 * BSM_EPATTERN, BSM_ENOMEM. */
int bsm_batch_create(bsm_ctx ctx, int n, const bsm_matrix *A, const bsm_matrix *B, const bsm_matrix *C,
                     const double *alpha, const double *beta, int precision, bsm_batch *out);
/* Queue the batch on the context stream; cfg NULL = the tuned (or default) schedule. */
int bsm_batch_run(bsm_batch batch, const bsm_batch_config *cfg);
/* Time every candidate schedule -- the separate launches, and for each of the
 * two persistent modes 3 orders x {1, 8} queues x {4, 8, 16} waves per CU (the
 * per-b mode only when it differs from one launch) -- `reps` timed runs each
 * after one warm-up run of the candidate, keep the fastest; so the tuned
 * schedule is never slower than separate launches by more than the timing
 * noise.  Synchronises. */
int bsm_batch_tune(bsm_batch batch, int reps, bsm_batch_config *best, double *best_ms);
int bsm_batch_flops(bsm_batch batch, double *flops);
int bsm_batch_destroy(bsm_batch batch);

/* Algorithmic flops of mask_{P_C}(A B): 2 b^3 per block triple (i, k, j). */
int bsm_product_flops(bsm_ctx ctx, bsm_pattern PA, bsm_pattern PB, bsm_pattern PC, double *flops);

/* *out = Tr(A B) = sum over (i,k) in P_A of sum_pq A_ik[p][q] B_ki[q][p], in FP64,
 * blocks missing from P_B counting as zero.  Deterministic (fixed reduction
 * order).  Synchronises.  Errors: BSM_EPATTERN, BSM_ENONFINITE (result not
 * finite; *out is still written). */
int bsm_trace_product(bsm_ctx ctx, const bsm_matrix *A, const bsm_matrix *B, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): Tr(A B) as
 * bsm_trace_product computes it (same kernels and reduction order, so the same
 * bits), written to out_dev, one double in DEVICE memory, asynchronously on the
 * context stream.  The per-workgroup partial sums live in a static device array
 * of the library (1032 doubles = 8256 bytes per GPU, held until the process
 * ends), whose address bsm_ctx_create takes once per device; the call itself
 * allocates nothing, copies nothing to the host and does not synchronise, so
 * it reports no BSM_ENONFINITE (a non-finite trace is written as it is).  The
 * number of partial sums is fixed by the reduction grid (at most 1024), so no
 * input size exceeds the scratch.  All calls on one GPU share that array:
 * calls that overlap in time on one GPU (other streams, other contexts, other
 * threads) race and give wrong results; calls ordered on one stream are safe.
 * Errors: BSM_EINVAL (NULL argument, non-FP64 matrix), BSM_EPATTERN, BSM_EHIP. */
int bsm_trace_product_noalloc(bsm_ctx ctx, const bsm_matrix *A, const bsm_matrix *B, double *out_dev);

/* ---- Hotelling iteration for S^-1 (paper: linear-scaling inversion of the
 *      overlap matrix, Development Priorities) ---------------------------- */
typedef struct {
    int max_iter;        /* maximum number of updates */
    double tol;          /* stop when ||I - Z S||_F < tol sqrt(N_b); <= 0: run max_iter */
    int init_given;      /* 0: Z0 = I / rho (rho = largest absolute row sum of S);
                            1: start from Z's current contents;
                            2: guarded correction: Z holds dZ; start from
                               I / rho + dZ when its residual is finite and below
                               that of I / rho, else from I / rho; a corrected
                               start that diverges or stops above 0.1 sqrt(N_b)
                               is rerun from I / rho */
} hot_params;

typedef struct {
    int status;          /* BSM_OK, BSM_EDIVERGED, BSM_ENOTCONV or BSM_ENONFINITE */
    int iterations;      /* updates accepted */
    double alpha;        /* 1 / rho (0 when init_given == 1) */
    double *residuals;   /* host, caller-owned, capacity entries (may be NULL) */
    int capacity;
    int n_residuals;     /* residual of Z0 and of every accepted update */
    double product_flops; /* algorithmic flops of the products launched */
    int start;           /* 0: the iteration ran from I / rho; 1: from Z's contents */
} hot_result;

/* Truncated Hotelling / Schulz iteration Z <- sym(mask_Z(2Z - (Z S) Z)) on Z's
 * pattern, with T = Z S held exactly on P(r_Z + r_S) and the residual
 * ||I - Z S||_F summed elementwise over T - I (a deterministic reduction).  Stops at
 * the tolerance, at max_iter, or when an update makes no real progress (the
 * next residual is above 0.99 times the current one: the current Z is kept; accepted when its residual is
 * at most 0.1 sqrt(N_b), the truncation floor, else BSM_EDIVERGED, which a
 * growing residual from an indefinite S always gives).  S and Z must be built
 * from the same positions.  Returns the
 * same code as result->status, except BSM_ENOTCONV, which returns BSM_OK with
 * Z valid. */
int hotelling_inverse(bsm_ctx ctx, const bsm_matrix *S, const bsm_matrix *Z,
                      const hot_params *params, hot_result *result);

/* Inverse square root of the overlap matrix (the companion of its inversion,
 * Development Priorities, for symmetric orthogonalisation): the coupled
 * Newton-Schulz iteration (Higham 1997) on A = S / rho, rho the largest
 * absolute row sum of S: Y0 = mask_Z(A), Z0 = I, then per update
 * P = Z Y, T = (3 I - P) / 2, Y <- sym(mask_Z(Y T)), Z <- sym(mask_Z(T Z)),
 * with P and T held exactly on P(2 r_Z) and the residual ||I - Z Y||_F summed
 * elementwise over P - I.  Stops as hotelling_inverse (tolerance, max_iter, no
 * real progress: accepted at or below 0.1 sqrt(N_b), else BSM_EDIVERGED).
 * On return Z holds S^-1/2 = Z_k / sqrt(rho) and, when Y is not NULL,
 * Y holds S^1/2 = sqrt(rho) Y_k, both on Z's pattern (Y must be built on the
 * same pattern object).  params->init_given must be 0; result->alpha = 1 / rho.
 * S, Z and Y must not alias.  Returns as hotelling_inverse (BSM_ENOTCONV is
 * returned as BSM_OK with the outputs valid); BSM_EPATTERN if Y is on another
 * pattern. */
int bsm_inverse_sqrt(bsm_ctx ctx, const bsm_matrix *S, const bsm_matrix *Z, const bsm_matrix *Y,
                     const hot_params *params, hot_result *result);

/* ---- LNV density-matrix minimisation (paper: the linear-scaling O(N)
 *      solver, Background; its full GPU form, Meeting the Exascale Challenges) */
enum { LNV_CANONICAL = 0, LNV_GRAND = 1 };

typedef struct {
    double n_electrons;  /* N_e (spin-paired: E = 2 Tr KH, N = 2 Tr KS) */
    int mode;            /* LNV_CANONICAL: mu from the gradients, N held at N_e;
                            LNV_GRAND: fixed mu, no projection */
    double mu;           /* fixed chemical potential for LNV_GRAND */
    double tol_E;        /* converged when |E_n - E_(n-1)| < tol_E (Ha) */
    int init_from_z;     /* 1: L <- c mask_L(Z) with N(c Z) = N_e; 0: use L as given */
    int product_precision; /* BSM_F64 (default 0), BSM_F32 or BSM_BF16 for every product
                              of a step (bsm_multiply_truncate_prec); traces stay FP64 */
} lnv_params;

typedef struct {
    double E, Omega, N, mu;   /* at the L this step started from */
    double alpha;             /* line-search step taken */
    double beta;              /* conjugate-gradient coefficient used */
    double dE;                /* E - E_previous (NaN on the first step) */
    double c[4];              /* Omega(alpha) = c0 + c1 a + c2 a^2 + c3 a^3 */
    int converged;
    int status;
    double product_flops;     /* algorithmic flops of this step's products */
} lnv_result;

typedef struct lnv_state_s lnv_state;

/* Create a minimisation over L's pattern P_L.  S and H share one pattern; Z is
 * the (truncated) S^-1 from hotelling_inverse.  L is caller-owned and is
 * updated in place by every step.  Scratch (eight matrices on P(r_L + r_S),
 * one on P(r_Z + r_L), twelve on P_L) comes from the context allocator; the
 * wider patterns are built once per context and reused.
 * Errors: BSM_EPATTERN, BSM_EINVAL, BSM_ENOMEM, BSM_ENONFINITE. */
int lnv_state_create(bsm_ctx ctx, const bsm_matrix *S, const bsm_matrix *H, const bsm_matrix *Z,
                     const bsm_matrix *L, const lnv_params *params, lnv_state **out);
/* One conjugate-gradient iteration with an exact cubic line search:
 * X = LS, Y = LH, W = XX, U = YX on P(r_L + r_S); E = 2(3 Tr XY - 2 Tr WY),
 * N = 2(3 Tr XX - 2 Tr WX); gradients G_E, G_N on P_L; preconditioning
 * M(G) = mask_L(Z G Z); Polak-Ribiere direction; Omega(alpha) cubic from
 * traces; L <- sym(L + alpha D + delta M(G_N)) with delta restoring N_e.
 * Returns result->status. */
int lnv_step(lnv_state *st, lnv_result *result);
/* Start over with new parameters on the same matrices (after Z or L changed):
 * clears the conjugate-gradient history and, with init_from_z, recomputes
 * L0 = c mask_L(Z).  *init_flops (may be NULL) receives the algorithmic flops of
 * the two products that takes.  Patterns and product plans are kept. */
int lnv_state_reset(lnv_state *st, const lnv_params *params, double *init_flops);
int lnv_state_destroy(lnv_state *st);

/* Idempotency diagnostic of the current L: with KS = 3 W - 2 mask_X(W X) on
 * P_X = P(r_L + r_S) (W = X X, X = L S; the truncated form of K S for
 * K = 3LSL - 2LSLSL), *e_idem = ||mask_X(KS KS) - KS||_F / ||KS||_F, which
 * vanishes when K S K = K.  FP64 products; overwrites the state's P_X scratch
 * (harmless: every step recomputes it).  Synchronises. */
int lnv_idempotency_error(lnv_state *st, double *e_idem);

/* Forces at the current L (meant for a converged L: the paper lists forces with
 * the solver's next capabilities; the standard derivative of the density-matrix
 * functional): F_I = -d Omega / d R_I, Omega = E - mu (N - N_e), at fixed L,
 *     F_I^c = 4 sum_{j != I} <K_Ij, dH^c_Ij> + <(Q - mu K)_Ij, dS^c_Ij>   (elementwise)
 * with K = 3LSL - 2LSLSL, H' = H - mu S and the energy-density matrix
 * Q = 3 L H' L - 2 (LSL H' L + L H' LSL), both on P_S, and mu from the current
 * gradients (<G_N, M(G_E)> / <G_N, M(G_N)>; the state's mu in LNV_GRAND mode).
 * dS and dH are arrays of 3 matrices (x, y, z) on the state's S and H pattern
 * objects holding, for every block (i, j), d(block)/dR_j (d/dR_i is its negative;
 * diagonal blocks are ignored).  S and H must share one pattern range.  forces:
 * host, natoms x 3 doubles (caller-owned); mu: optional host output.  FP64
 * products; overwrites the state's P_X scratch (every step recomputes it).
 * Synchronises.  Errors: BSM_EPATTERN (derivative patterns), BSM_ENONFINITE. */
int lnv_forces(lnv_state *st, const bsm_matrix *dS, const bsm_matrix *dH, double *forces, double *mu);

/* A precision schedule for a whole solve (an extension built on the method: low-precision
 * products with FP64 traces, then FP64 refinement).  Stage s runs lnv_step with
 * products in precision[s] until |dE| < tol_E[s] (tol_E[s] > 0), or, when
 * stop_on_rise[s], until E fails to decrease (the rounding floor of that
 * precision), or max_iter[s] steps.  The first stage continues the state as
 * created or reset; each later stage keeps L and restarts the conjugate
 * gradients.  A last stage with tol_E = 0 runs exactly max_iter FP64 steps. */
#define LNV_MAX_STAGES 4
typedef struct {
    int n_stages;
    int precision[LNV_MAX_STAGES];
    int max_iter[LNV_MAX_STAGES];
    double tol_E[LNV_MAX_STAGES];
    int stop_on_rise[LNV_MAX_STAGES];
} lnv_schedule;

typedef struct {
    int status;                      /* BSM_OK or the failing step's status */
    int converged;                   /* last stage met its stop rule (tol or count) */
    int iterations[LNV_MAX_STAGES];  /* steps taken per stage */
    double E, N, mu;                 /* last step's values (at the L it started from) */
    double product_flops;            /* algorithmic flops of all products */
} lnv_solve_result;

int lnv_solve(lnv_state *st, const lnv_schedule *schedule, lnv_solve_result *result);

#ifdef __cplusplus
}
#endif
#endif /* BSM_H */
