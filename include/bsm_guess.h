/*
 * bsm_guess.h -- C ABI of the learned initial guess for the Hotelling and LNV
 * drivers of bsm.h (an extension: the paper lists machine-learned methods
 * among the code's development directions, section "Development Priorities",
 * but fixes no model).
 *
 * A three-layer perceptron maps a 32-value descriptor of every atom pair of a
 * pattern to a correction of that pair's block in the method's own starting
 * points,
 *     Z0 = alpha I + scale * dZ   (Hotelling, alpha = 1 / max abs row sum of S)
 *     L0 = c mask_L(Z) + scale * dL   (LNV, c from N(c Z) = N_e),
 * so a network whose last layer is zero gives back the plain starts, and the
 * drivers keep the plain start whenever the corrected one is worse (guarded
 * starts below).  The network is trained on the GPU, by the kernels of this
 * library, on solves the library itself produced.
 *
 * Conventions are those of bsm.h (status codes, device / host pointers,
 * stream ordering, one host thread per context).
 *
 * Descriptor of the pattern slot (i, j), r = minimum-image vector from atom i
 * to atom j, d = |r|, r_c = the pattern's cutoff, rhat = r / d (0 when i = j):
 *     [0..2] r / r_c   [3] d / r_c   [4] (d / r_c)^2   [5] exp(-d / 1.5 A)
 *     [6] s_i   [7] s_j   [8..11] rhat . e_i[a]   [12..15] rhat . e_j[a]
 *     [16..19] 10 (l_i[a] - d0)   [20..23] 10 (l_j[a] - d0)
 *     [24..26] 10 c_i   [27..29] 10 c_j   [30, 31] 0
 * (lengths in Angstrom) where, from the four nearest neighbours of an atom
 * (ordered by squared distance, then index) with vectors w_n, unit vectors
 * v_n and the tetrahedral directions T_a = (+-1, +-1, +-1) / sqrt 3 of
 * diamond's first sublattice,
 *     s = +1 if sum_n max_a v_n . T_a >= sum_n max_a (-v_n . T_a), else -1,
 *     e[a] = the v_n with the largest s v_n . T_a (first n on ties), l[a] its |w_n|,
 *     c = (w_1 + w_2 + w_3 + w_4) / 4,
 * and d0 = 5.43 sqrt(3) / 4 A, the ideal Si-Si bond: features 16..29 measure
 * the local strain of the two atoms and vanish on the ideal lattice.
 *
 * Network: h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3 with
 * x of 32 values, width H = 128, M outputs (b^2 for blocks of b orbitals).
 * Parameters are one FP32 array in the order W1 (32 x H), b1 (H), W2 (H x H),
 * b2 (H), W3 (H x M), b3 (M), every weight matrix row-major with the input
 * index first.  Minibatch loss: (1 / 2n) sum over samples and outputs of
 * (y - t)^2.  Optimiser: Adam with bias correction (Kingma, Ba 2015).
 */
#ifndef BSM_GUESS_H
#define BSM_GUESS_H

#include "bsm.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { BSM_DESC_DIM = 32, BSM_MLP_WIDTH = 128 };

typedef struct bsm_mlp_s *bsm_mlp;

typedef struct {
    int width;     /* hidden width: 128 */
    int out_dim;   /* outputs per sample, 1..128 (b^2) */
} bsm_mlp_shape;

typedef struct {
    float lr, beta1, beta2, eps;   /* Adam step size, moment decays, denominator guard */
} bsm_adam;

typedef struct {
    int epochs;
    int batch;       /* samples per minibatch (one Adam step each), >= 1 */
    bsm_adam opt;
} bsm_mlp_train_params;

/* Number of FP32 parameters of a network of this shape; negative if the shape
 * is not supported. */
int64_t bsm_mlp_param_count(const bsm_mlp_shape *shape);
/* Create a network with the given parameters (host, param_count floats; the
 * caller draws them: the library draws no random numbers).  Adam's moments
 * start at zero.  Errors: BSM_EINVAL (shape), BSM_ENOMEM. */
int bsm_mlp_create(bsm_ctx ctx, const bsm_mlp_shape *shape, const float *params, bsm_mlp *out);
/* Copy the parameters to / from host memory; set also clears Adam's state.  Synchronise. */
int bsm_mlp_get_params(bsm_mlp net, float *params);
int bsm_mlp_set_params(bsm_mlp net, const float *params);
int bsm_mlp_destroy(bsm_mlp net);

/* Descriptors of every slot of P, in slot order: desc is device memory of
 * nnzb(P) x 32 floats.  Atom frames come from the four nearest neighbours in
 * `neighbours` (a pattern over the same positions whose every row holds at
 * least four atoms besides the diagonal, e.g. the overlap pattern).  Per slot
 * (i, j) with minimum-image vector r, d = |r|, cutoff r_c of P: r / r_c, d / r_c,
 * (d / r_c)^2, exp(-d / 1.5 A), the sublattice signs of i and j, the cosines of r
 * with the four bond directions of i and of j, 10 (bond length - ideal) of
 * those bonds for i and j, 10 x the neighbour centroids of i and j, and
 * 10 (rho - rho_0) for i and j, rho the sum of exp(-d / 1.5 A) over the atom's
 * row of `neighbours` (its environment) and rho_0 its value for an ideal-lattice
 * atom over a 6 A pattern.  Values are computed in FP64 and rounded to FP32.
 * desc must be 16-byte aligned.
 * Errors: BSM_EPATTERN (different atoms), BSM_EINVAL (a row with fewer than
 * four neighbours, misaligned desc). */
int bsm_pair_descriptors(bsm_ctx ctx, bsm_pattern neighbours, bsm_pattern P, float *desc);

/* Y (device, n x M floats) = network(X) for X (device, n x 32 floats, 16-byte
 * aligned).
 * precision BSM_F32: FP32 arithmetic throughout; BSM_BF16: inputs,
 * activations and weights rounded to BF16 (nearest, ties to even) on the
 * matrix cores with FP32 accumulation, bias and tanh in FP32. */
int bsm_mlp_forward(bsm_mlp net, int precision, int64_t n, const float *X, float *Y);
/* Minibatch loss (host, FP64 sum of FP32 terms) and its gradient (device,
 * param_count floats) in FP32, for samples X (n x 32) and targets T (n x M).
 * Deterministic: fixed-order reductions. */
int bsm_mlp_loss_grad(bsm_mlp net, int64_t n, const float *X, const float *T, double *loss, float *grad);
/* One Adam step with the given gradient (device); the step counter is the
 * network's own. */
int bsm_mlp_adam_step(bsm_mlp net, const bsm_adam *opt, const float *grad);
/* Epochs of minibatch training: minibatch k of every epoch holds samples
 * perm[k batch .. (k + 1) batch - 1] (perm: device, n int32 indices into X
 * and T, each in [0, n): the kernels trust them; NULL = identity), one Adam
 * step each.  X and T must be 16-byte aligned.  epoch_loss (host, epochs
 * doubles, may be NULL) receives the mean minibatch loss of every epoch.
 * Synchronises once per epoch. */
int bsm_mlp_train(bsm_mlp net, const bsm_mlp_train_params *p, int64_t n, const float *X, const float *T,
                  const int32_t *perm, double *epoch_loss);

/* Training targets from two matrices on one pattern: T (device, nnzb x b^2
 * floats) = (A - B) / scale, slot by slot. */
int bsm_mlp_targets(bsm_ctx ctx, const bsm_matrix *A, const bsm_matrix *B, double scale, float *T);
/* M <- beta M + scale * network(X) block by block, X the descriptors of M's
 * pattern (device, nnzb x 32); the network's out_dim must be b^2.  beta == 0
 * ignores M's old contents. */
int bsm_mlp_predict_blocks(bsm_mlp net, int precision, const float *X, double scale, double beta,
                           const bsm_matrix *M);

/* Guarded LNV start.  Forms the plain start L_p = c mask_L(Z) (as
 * lnv_state_reset with init_from_z), then the corrected L_g = L_p + dL (dL on
 * L's pattern), evaluates E and N of both and keeps L_g only when both are
 * finite, |N_g - N_e| <= n_tol N_e and E_g < E_p; otherwise L_p.  Clears the
 * conjugate-gradient history as lnv_state_reset does. */
typedef struct {
    int accepted;            /* 1: L holds L_g; 0: L holds L_p */
    double E_plain, N_plain;
    double E_guess, N_guess;
    double product_flops;    /* algorithmic flops of the products taken */
} lnv_guess_result;
int lnv_state_reset_guess(lnv_state *st, const lnv_params *params, const bsm_matrix *dL, double n_tol,
                          lnv_guess_result *out);

#ifdef __cplusplus
}
#endif
#endif
