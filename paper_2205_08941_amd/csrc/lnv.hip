// LNV density-matrix minimisation on the GPU.
//
// The paper's linear-scaling solver finds the ground-state density matrix by
// minimisation over a truncated auxiliary matrix (Background and Current
// Status) and names a full GPU implementation of it as the goal (Meeting the
// Exascale Challenges).  Here that is the non-orthogonal LNV functional
// (Li, Nunes, Vanderbilt 1993; Nunes, Vanderbilt 1994):
//   K = 3 LSL - 2 LSLSL,  E = 2 Tr KH,  N = 2 Tr KS,  Omega = E - mu N,
// minimised over L in span(P_L) by Polak-Ribiere conjugate gradients with the
// S^-1-preconditioned gradient M(G) = mask_L(Z G Z), mu from the gradients so
// that the search direction keeps N fixed to first order, an exact line search
// (Omega is cubic along any line) and a first-order correction back to N_e.
// Every intermediate is held on a pattern wide enough for the blocks later
// steps read, so E, N and their gradients are exact for the truncated L.
#include "bsm_internal.h"
#include "bsm_guess.h"

#include <cmath>
#include <functional>

namespace bsm {
namespace {

struct Mat {
    const bsm_pattern_s *p = nullptr;
    DevBuf buf;
    Mat() = default;
    Mat(Context *c, const bsm_pattern_s *pat) : p(pat), buf(c, sizeof(double) * (size_t)std::max<int64_t>(1, nelems(pat))) {}
    double *d() const { return buf.as<double>(); }
    int64_t n() const { return nelems(p); }
};

double newton(const std::function<double(double)> &f, const std::function<double(double)> &df, double x)
{
    for (int it = 0; it < 100; ++it) {
        const double step = f(x) / df(x);
        x -= step;
        if (std::fabs(step) <= 1e-16 * std::max(1.0, std::fabs(x))) break;
    }
    return x;
}

// c with N(c Z) = 2 (3 c^2 t2 - 2 c^3 t3) = N_e nearest c0, 3 c0^2 - 2 c0^3 = N_e / (2 N_b)
double initial_scale(double nb, double ne, double t2, double t3)
{
    const double nu = ne / (2.0 * nb);
    const double c0 = newton([&](double c) { return 3 * c * c - 2 * c * c * c - nu; },
                             [&](double c) { return 6 * c - 6 * c * c; }, 0.5);
    return newton([&](double c) { return 2 * (3 * c * c * t2 - 2 * c * c * c * t3) - ne; },
                  [&](double c) { return 2 * (6 * c * t2 - 6 * c * c * t3); }, c0);
}

// Row sums of the force terms: one workgroup per atom I, out[3 I + c] =
// 4 sum over the off-diagonal blocks s of row I of <K_s, dH^c_s> + <Wt_s, dS^c_s>
// (elementwise), in a fixed order (strided partial sums, then a fixed tree).
constexpr int kForceThreads = 256;
__global__ __launch_bounds__(kForceThreads) void k_row_forces(int b, const int *__restrict__ rowptr,
                                                              const int *__restrict__ cols,
                                                              const double *__restrict__ K,
                                                              const double *__restrict__ Wt,
                                                              const double *__restrict__ dH0,
                                                              const double *__restrict__ dH1,
                                                              const double *__restrict__ dH2,
                                                              const double *__restrict__ dS0,
                                                              const double *__restrict__ dS1,
                                                              const double *__restrict__ dS2, double *__restrict__ out)
{
    __shared__ double red[3][kForceThreads];
    const int I = blockIdx.x, bb = b * b;
    const int s0 = rowptr[I], s1 = rowptr[I + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t e = (int64_t)s0 * bb + threadIdx.x; e < (int64_t)s1 * bb; e += kForceThreads) {
        if (cols[e / bb] == I) continue;   // a block of the atom with itself does not move
        const double k = K[e], w = Wt[e];
        a0 += k * dH0[e] + w * dS0[e];
        a1 += k * dH1[e] + w * dS1[e];
        a2 += k * dH2[e] + w * dS2[e];
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    __syncthreads();
    for (int w = kForceThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[3 * I + threadIdx.x] = 4.0 * red[threadIdx.x][0];
}

}  // namespace
}  // namespace bsm

using namespace bsm;

struct lnv_state_s {
    Context *c = nullptr;
    const bsm_pattern_s *PS = nullptr, *PH = nullptr, *PZ = nullptr, *PL = nullptr;
    const double *S = nullptr, *H = nullptr, *Z = nullptr;
    double *L = nullptr;
    const bsm_pattern_s *PX = nullptr, *PZG = nullptr;   // owned by the context's cache
    lnv_params prm{};
    double mu = 0.0;
    int n = 0;
    double E_prev = NAN;
    bool have_prev = false;
    // P_X: X, Y, W, U (reused for X + X_D), X_D, Y_D, Q, W1 (reused for M1)
    Mat X, Y, W, U, XD, YD, Q, W1;
    Mat ZG;
    // P_L
    Mat GE, GN, PE, PN, g, Mg, D, Dprev, gprev, Mgprev, t1, t2;
    double flops = 0.0;

    int prec = BSM_F64;   // precision of the step's products

    void mul(double alpha, const bsm_pattern_s *pa, const double *a, const bsm_pattern_s *pb, const double *b,
             double beta, const bsm_pattern_s *pc, double *cc)
    {
        Plan *plan = get_plan(c, pa, pb, pc);
        launch_product_mixed(c, plan, prec, alpha, pa, a, pb, b, beta, pc, cc);
        flops += plan->flops;
    }
    void mul(const Mat &A, const Mat &B, Mat &C) { mul(1.0, A.p, A.d(), B.p, B.d(), 0.0, C.p, C.d()); }
    // C = A B and C2 = A2 B (A, A2 on one pattern, C, C2 on one pattern): FP64 pairs share B's
    // copies in one launch with the same results as two products
    void mul_pair(const bsm_pattern_s *pa, const double *a, const double *a2, const bsm_pattern_s *pb,
                  const double *b, const bsm_pattern_s *pc, double *c1, double *c2)
    {
        Plan *pair = prec == BSM_F64 ? get_pair_plan(c, pa, pb, pc) : nullptr;
        if (!pair) {
            mul(1.0, pa, a, pb, b, 0.0, pc, c1);
            mul(1.0, pa, a2, pb, b, 0.0, pc, c2);
            return;
        }
        launch_product_pair_f64(c, pair, 1.0, pa, a, a2, pb, b, 0.0, pc, c1, c2);
        flops += 2.0 * pair->flops;
    }
    void mul_pair(const Mat &A, const Mat &A2, const Mat &B, Mat &C, Mat &C2)
    {
        mul_pair(A.p, A.d(), A2.d(), B.p, B.d(), C.p, C.d(), C2.d());
    }
    // C = A S and C2 = A H (the left operand shared): one launch when H and S lie on one pattern
    void mul_pair_sh(const bsm_pattern_s *pa, const double *a, const bsm_pattern_s *pc, double *c1, double *c2)
    {
        Plan *pair = prec == BSM_F64 && PH == PS ? get_pair_plan_a(c, pa, PS, pc) : nullptr;
        if (!pair) {
            mul(1.0, pa, a, PS, S, 0.0, pc, c1);
            mul(1.0, pa, a, PH, H, 0.0, pc, c2);
            return;
        }
        launch_product_pair_a_f64(c, pair, 1.0, pa, a, PS, S, H, 0.0, pc, c1, c2);
        flops += 2.0 * pair->flops;
    }
    void precondition(const Mat &G, Mat &out)
    {
        mul(1.0, PZ, Z, G.p, G.d(), 0.0, ZG.p, ZG.d());
        mul(1.0, ZG.p, ZG.d(), PZ, Z, 0.0, out.p, out.d());
        symmetrize(c, out.p, out.d());
    }
    // Clear the conjugate-gradient history; with init_from_z, L0 = c mask_L(Z) where
    // t_m = Tr[(Z S)^m] (T = Z S exact on P(r_Z + r_S)) and N(c Z) = N_e.
    void reset(const lnv_params &p)
    {
        BSM_REQUIRE(p.product_precision == BSM_F64 || p.product_precision == BSM_F32 ||
                        p.product_precision == BSM_BF16,
                    BSM_EINVAL, "bad product precision");
        prm = p;
        mu = p.mu;
        n = 0;
        E_prev = NAN;
        have_prev = false;
        init_flops = 0.0;
        prec = BSM_F64;   // the initial guess is always formed in FP64
        if (!p.init_from_z) {
            prec = p.product_precision;
            return;
        }
        const bsm_pattern_s *PT = derived_pattern_cached(PZ, PZ->cutoff + PS->cutoff);
        // T and T2 live in the X and Y buffers when they fit (they are free until the first
        // energy evaluation): no extra device memory next to the state, which at 32768 atoms
        // would not fit beside it
        Mat Tm, T2m;
        double *tb = X.d(), *t2b = Y.d();
        if (nelems(PT) > X.n()) {
            Tm = Mat(c, PT);
            T2m = Mat(c, PT);
            tb = Tm.d();
            t2b = T2m.d();
        }
        flops = 0.0;
        mul(1.0, PZ, Z, PS, S, 0.0, PT, tb);
        mul(1.0, PT, tb, PT, tb, 0.0, PT, t2b);
        init_flops = flops;
        const double *a[2] = {tb, t2b}, *b[2] = {tb, tb};
        double tt[2];
        trace_products(c, 2, PT, a, PT, b, tt);
        BSM_REQUIRE(std::isfinite(tt[0]) && std::isfinite(tt[1]), BSM_ENONFINITE, "initial traces are not finite");
        const double nb = (double)PL->natoms * PL->b;
        const double scale = initial_scale(nb, p.n_electrons, tt[0], tt[1]);
        mask_copy(c, PZ, Z, PL, L);
        axpby(c, nelems(PL), scale, L, 0.0, L);
        BSM_HIP_TRY(hipStreamSynchronize(c->stream));
        prec = p.product_precision;
    }
    int step(lnv_result *res);
    double init_flops = 0.0;

    // E = 2 Tr KH and N = 2 Tr KS of the current L (X = LS, Y = LH, W = XX on P_X)
    void energy(double &E, double &N)
    {
        mul_pair_sh(PL, L, X.p, X.d(), Y.d());                   // X = L S, Y = L H
        mul(X, X, W);
        double tr[4];   // Tr XY, Tr WY, Tr XX, Tr WX
        const double *a[2] = {X.d(), W.d()}, *b[2] = {Y.d(), X.d()};
        trace_set(c, kTracesEnergy, X.p, a, b, tr);
        E = 2.0 * (3.0 * tr[0] - 2.0 * tr[1]);
        N = 2.0 * (3.0 * tr[2] - 2.0 * tr[3]);
    }

    // G_E = sym(6 (HX + (HX)^T) - 4 (HW + (HW)^T) - 4 S U), G_N = sym(12 (S X - S W)) on P_L
    // from X, W, U of the current L
    void gradients()
    {
        const int64_t nl = nelems(PL);
        if (PH == PS) {
            // H and S on one pattern: HX with SX and HW with SW as paired launches (B's copies
            // shared); the same sums in the same order as below (PE is free until preconditioning)
            mul_pair(PH, H, S, X.p, X.d(), PL, t1.d(), t2.d());      // HX, SX
            add_transpose(c, PL, 6.0, t1.d(), 0.0, GE.d());        // 6 (HX + HX^T)
            mul_pair(PH, H, S, W.p, W.d(), PL, t1.d(), PE.d());      // HW, SW
            add_transpose(c, PL, -4.0, t1.d(), 1.0, GE.d());       // - 4 (HW + HW^T)
            mul(1.0, PS, S, U.p, U.d(), 0.0, PL, t1.d());          // SU
            axpby(c, nl, -4.0, t1.d(), 1.0, GE.d());               // - 4 SU
            symmetrize(c, PL, GE.d());
            axpbypcz(c, nl, 12.0, t2.d(), -12.0, PE.d(), 0.0, GN.d());
            symmetrize(c, PL, GN.d());
            return;
        }
        mul(1.0, PH, H, X.p, X.d(), 0.0, PL, t1.d());          // HX
        add_transpose(c, PL, 6.0, t1.d(), 0.0, GE.d());        // 6 (HX + HX^T)
        mul(1.0, PH, H, W.p, W.d(), 0.0, PL, t1.d());          // HW
        add_transpose(c, PL, -4.0, t1.d(), 1.0, GE.d());       // - 4 (HW + HW^T)
        mul(1.0, PS, S, U.p, U.d(), 0.0, PL, t1.d());          // SU
        axpby(c, nl, -4.0, t1.d(), 1.0, GE.d());               // - 4 SU
        symmetrize(c, PL, GE.d());
        mul(1.0, PS, S, X.p, X.d(), 0.0, PL, t1.d());          // SX
        mul(1.0, PS, S, W.p, W.d(), 0.0, PL, t2.d());          // SW
        axpbypcz(c, nl, 12.0, t1.d(), -12.0, t2.d(), 0.0, GN.d());
        symmetrize(c, PL, GN.d());
    }

    double dot1(const Mat &A, const Mat &B)
    {
        const double *a = A.d(), *b = B.d();
        double r = 0.0;
        dots(c, 1, A.p, &a, &b, &r);
        return r;
    }
};

extern "C" int lnv_state_create(bsm_ctx ctx, const bsm_matrix *S, const bsm_matrix *H, const bsm_matrix *Z,
                                const bsm_matrix *L, const lnv_params *prm, lnv_state **out)
{
    try {
        BSM_REQUIRE(ctx && prm && out, BSM_EINVAL, "NULL argument");
        check_matrix(S, "S");
        check_matrix(H, "H");
        check_matrix(Z, "Z");
        check_matrix(L, "L");
        check_same_shape(S, H);
        check_same_shape(S, Z);
        check_same_shape(S, L);
        BSM_REQUIRE(prm->mode == LNV_CANONICAL || prm->mode == LNV_GRAND, BSM_EINVAL, "bad mode");
        Context *c = &ctx->c;
        std::unique_ptr<lnv_state_s> st(new lnv_state_s());
        st->c = c;
        st->PS = S->pattern;
        st->PH = H->pattern;
        st->PZ = Z->pattern;
        st->PL = L->pattern;
        st->S = (const double *)S->blocks;
        st->H = (const double *)H->blocks;
        st->Z = (const double *)Z->blocks;
        st->L = (double *)L->blocks;
        st->prm = *prm;
        st->mu = prm->mu;
        const double rx = st->PL->cutoff + std::max(st->PS->cutoff, st->PH->cutoff);
        st->PX = derived_pattern_cached(st->PL, rx);
        st->PZG = derived_pattern_cached(st->PL, st->PZ->cutoff + st->PL->cutoff);
        const bsm_pattern_s *PX = st->PX, *PL = st->PL;
        for (Mat *m : {&st->X, &st->Y, &st->W, &st->U, &st->XD, &st->YD, &st->Q, &st->W1}) *m = Mat(c, PX);
        st->ZG = Mat(c, st->PZG);
        for (Mat *m : {&st->GE, &st->GN, &st->PE, &st->PN, &st->g, &st->Mg, &st->D, &st->Dprev, &st->gprev,
                       &st->Mgprev, &st->t1, &st->t2})
            *m = Mat(c, PL);
        st->reset(*prm);
        *out = st.release();
        return BSM_OK;
    } catch (const Error &e) {
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}

extern "C" int lnv_state_reset(lnv_state *st, const lnv_params *prm, double *init_flops)
{
    try {
        BSM_REQUIRE(st && prm, BSM_EINVAL, "NULL argument");
        BSM_REQUIRE(prm->mode == LNV_CANONICAL || prm->mode == LNV_GRAND, BSM_EINVAL, "bad mode");
        st->reset(*prm);
        if (init_flops) *init_flops = st->init_flops;
        return BSM_OK;
    } catch (const Error &e) {
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}

extern "C" int lnv_state_reset_guess(lnv_state *st, const lnv_params *prm, const bsm_matrix *dL, double n_tol,
                                     lnv_guess_result *out)
{
    try {
        BSM_REQUIRE(st && prm && dL && out, BSM_EINVAL, "NULL argument");
        BSM_REQUIRE(prm->mode == LNV_CANONICAL || prm->mode == LNV_GRAND, BSM_EINVAL, "bad mode");
        BSM_REQUIRE(n_tol >= 0.0, BSM_EINVAL, "n_tol must be >= 0");
        check_matrix(dL, "dL");
        BSM_REQUIRE(dL->pattern == st->PL, BSM_EPATTERN, "dL must be on L's pattern");
        BSM_REQUIRE(dL->blocks != st->L, BSM_EINVAL, "dL aliases L");
        *out = lnv_guess_result{};
        lnv_params p = *prm;
        p.init_from_z = 1;
        st->reset(p);                       // L = c mask_L(Z) (formed with FP64 products)
        st->flops = 0.0;
        Context *c = st->c;
        const int64_t nl = nelems(st->PL);
        // both energies of the accept test with FP64 products, whatever the state's
        // product precision; that precision is restored on every exit
        struct PrecGuard {
            lnv_state_s *s;
            int p;
            ~PrecGuard() { s->prec = p; }
        } guard{st, prm->product_precision};
        st->prec = BSM_F64;
        st->energy(out->E_plain, out->N_plain);
        BSM_HIP_TRY(hipMemcpyAsync(st->t1.d(), st->L, sizeof(double) * nl, hipMemcpyDeviceToDevice, c->stream));
        axpby(c, nl, 1.0, (const double *)dL->blocks, 1.0, st->L);
        st->energy(out->E_guess, out->N_guess);
        out->accepted = std::isfinite(out->E_guess) && std::isfinite(out->N_guess) &&
                        std::fabs(out->N_guess - prm->n_electrons) <= n_tol * prm->n_electrons &&
                        out->E_guess < out->E_plain;
        if (!out->accepted)
            BSM_HIP_TRY(hipMemcpyAsync(st->L, st->t1.d(), sizeof(double) * nl, hipMemcpyDeviceToDevice, c->stream));
        BSM_HIP_TRY(hipStreamSynchronize(c->stream));
        out->product_flops = st->init_flops + st->flops;
        st->flops = 0.0;
        return BSM_OK;
    } catch (const Error &e) {
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}

extern "C" int lnv_state_destroy(lnv_state *st)
{
    if (st) {
        (void)hipStreamSynchronize(st->c->stream);
        delete st;
    }
    return BSM_OK;
}

extern "C" int lnv_step(lnv_state *st, lnv_result *res)
{
    try {
        BSM_REQUIRE(st && res, BSM_EINVAL, "NULL argument");
        return st->step(res);
    } catch (const Error &e) {
        if (res) res->status = e.code;
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}

int lnv_state_s::step(lnv_result *res)
{
    lnv_state_s *st = this;
    {
        Context *c = st->c;
        st->flops = 0.0;
        *res = lnv_result{};
        const bsm_pattern_s *PL = st->PL;
        const int64_t nl = nelems(PL), nx = nelems(st->PX);
        Mat &X = st->X, &Y = st->Y, &W = st->W, &U = st->U, &XD = st->XD, &YD = st->YD, &Q = st->Q, &W1 = st->W1;

        // ---- evaluate: X = LS, Y = LH, W = XX, U = YX; E, N from traces
        st->mul_pair_sh(PL, st->L, X.p, X.d(), Y.d());               // X = L S, Y = L H
        st->mul_pair(X, Y, X, W, U);                                 // W = X X, U = Y X
        double tr0[4];
        {
            const double *a[2] = {X.d(), W.d()}, *b[2] = {Y.d(), X.d()};   // Tr XY, Tr WY, Tr XX, Tr WX
            trace_set(c, kTracesEnergy, X.p, a, b, tr0);
        }
        const double E = 2.0 * (3.0 * tr0[0] - 2.0 * tr0[1]);
        const double N = 2.0 * (3.0 * tr0[2] - 2.0 * tr0[3]);
        res->E = E;
        res->N = N;
        res->mu = st->mu;
        if (!(std::isfinite(E) && std::isfinite(N))) {
            res->status = BSM_ENONFINITE;
            res->Omega = NAN;
            res->dE = NAN;
            return fail(BSM_ENONFINITE, "LNV energy is not finite");
        }

        // ---- gradients on P_L
        Mat &GE = st->GE, &GN = st->GN;
        st->gradients();

        // ---- preconditioned gradients, chemical potential, direction
        Mat &PE = st->PE, &PN = st->PN, &g = st->g, &Mg = st->Mg, &D = st->D;
        st->precondition(GE, PE);
        st->precondition(GN, PN);
        double gp[2];
        {
            const double *a[2] = {GN.d(), GN.d()}, *b[2] = {PN.d(), PE.d()};
            dots(c, 2, PL, a, b, gp);
        }
        const double gn_pn = gp[0];
        const bool canonical = st->prm.mode == LNV_CANONICAL && gn_pn > 0.0;
        const double mu = canonical ? gp[1] / gn_pn : st->mu;
        axpbypcz(c, nl, 1.0, GE.d(), -mu, GN.d(), 0.0, g.d());
        axpbypcz(c, nl, 1.0, PE.d(), -mu, PN.d(), 0.0, Mg.d());
        double beta = 0.0;
        if (st->n > 0 && st->n % 50 != 0 && st->have_prev) {
            const double den = st->dot1(st->gprev, st->Mgprev);
            axpbypcz(c, nl, 1.0, Mg.d(), -1.0, st->Mgprev.d(), 0.0, t1.d());
            beta = std::max(0.0, st->dot1(g, t1) / den);
        }
        // D = R + beta D_prev with R = -M(g)
        if (beta != 0.0) axpbypcz(c, nl, -1.0, Mg.d(), beta, st->Dprev.d(), 0.0, D.d());
        else axpby(c, nl, -1.0, Mg.d(), 0.0, D.d());
        if (st->dot1(g, D) >= 0.0) {
            beta = 0.0;
            axpby(c, nl, -1.0, Mg.d(), 0.0, D.d());
        }
        if (canonical) {
            const double proj = st->dot1(GN, D) / gn_pn;
            axpby(c, nl, -proj, PN.d(), 1.0, D.d());
        }

        // ---- exact line search along L + a D
        st->mul_pair_sh(PL, D.d(), XD.p, XD.d(), YD.d());            // X_D = D S, Y_D = D H
        st->mul(XD, XD, Q);                                          // Q = X_D X_D
        axpbypcz(c, nx, 1.0, X.d(), 1.0, XD.d(), 0.0, U.d());        // X1 = X + X_D (U is free now)
        st->mul(U, U, W1);                                           // W1 = X1 X1
        axpbypcz(c, nx, -1.0, W.d(), -1.0, Q.d(), 1.0, W1.d());      // M1 = W1 - W - Q = X X_D + X_D X
        Mat &M1 = W1;
        double tr[15];
        {
            // Tr of (X_D Y, X Y_D, X_D Y_D, X X_D, X_D X_D, M1 Y, W Y_D, Q Y, M1 Y_D, Q Y_D,
            //        M1 X, W X_D, Q X, M1 X_D, Q X_D)
            const double *a[5] = {XD.d(), X.d(), M1.d(), W.d(), Q.d()};
            const double *b[4] = {Y.d(), YD.d(), XD.d(), X.d()};
            trace_set(c, kTracesLineSearch, X.p, a, b, tr);
        }
        const double f[4] = {tr0[0], tr[0] + tr[1], tr[2], 0.0};
        const double h[4] = {tr0[2], 2.0 * tr[3], tr[4], 0.0};
        const double gg[4] = {tr0[1], tr[5] + tr[6], tr[7] + tr[8], tr[9]};
        const double kk[4] = {tr0[3], tr[10] + tr[11], tr[12] + tr[13], tr[14]};
        double e[4], nn[4], cc[4];
        for (int m = 0; m < 4; ++m) {
            e[m] = 2.0 * (3.0 * f[m] - 2.0 * gg[m]);
            nn[m] = 2.0 * (3.0 * h[m] - 2.0 * kk[m]);
            cc[m] = e[m] - mu * nn[m];
            res->c[m] = cc[m];
        }
        const double disc = cc[2] * cc[2] - 3.0 * cc[1] * cc[3];
        int status = BSM_OK;
        double den = 0.0;
        if (!(disc >= 0.0)) {
            status = BSM_ERUNAWAY;
        } else {
            den = cc[2] + std::sqrt(disc);
            if (!(den > 0.0)) status = BSM_ERUNAWAY;
        }
        const double dE = (st->n > 0) ? E - st->E_prev : NAN;
        res->Omega = E - mu * N;
        res->mu = mu;
        res->beta = beta;
        res->dE = dE;
        res->product_flops = st->flops;
        if (status != BSM_OK) {
            res->status = status;
            return fail(status, "LNV line search found no minimum (L left the basin)");
        }
        const double a = -cc[1] / den;
        double delta = 0.0;
        if (canonical) {
            const double Na = nn[0] + a * (nn[1] + a * (nn[2] + a * nn[3]));
            delta = (st->prm.n_electrons - Na) / gn_pn;
        }
        axpbypcz(c, nl, a, D.d(), delta, PN.d(), 1.0, st->L);
        symmetrize(c, PL, st->L);
        BSM_HIP_TRY(hipStreamSynchronize(c->stream));

        res->alpha = a;
        res->converged = (st->n > 0 && std::fabs(dE) < st->prm.tol_E) ? 1 : 0;
        res->status = BSM_OK;
        st->E_prev = E;
        st->mu = mu;
        std::swap(st->Dprev, st->D);
        std::swap(st->gprev, st->g);
        std::swap(st->Mgprev, st->Mg);
        st->have_prev = true;
        st->n += 1;
        return BSM_OK;
    }
}

extern "C" int lnv_idempotency_error(lnv_state *st, double *e_idem)
{
    try {
        BSM_REQUIRE(st && e_idem, BSM_EINVAL, "NULL argument");
        Context *c = st->c;
        const int saved = st->prec;
        st->prec = BSM_F64;
        const int64_t nx = nelems(st->PX);
        // X = L S, W = X X, then KS = 3 W - 2 mask_X(W X) and KS2 = mask_X(KS KS), all on P_X
        st->mul(1.0, st->PL, st->L, st->PS, st->S, 0.0, st->X.p, st->X.d());
        st->mul(st->X, st->X, st->W);
        st->mul(st->W, st->X, st->U);
        axpbypcz(c, nx, 3.0, st->W.d(), -2.0, st->U.d(), 0.0, st->Q.d());
        st->mul(st->Q, st->Q, st->W1);
        axpby(c, nx, -1.0, st->Q.d(), 1.0, st->W1.d());
        double d[2];
        const double *a[2] = {st->W1.d(), st->Q.d()}, *b[2] = {st->W1.d(), st->Q.d()};
        dots(c, 2, st->PX, a, b, d);
        st->prec = saved;
        *e_idem = std::sqrt(d[0]) / std::sqrt(d[1]);
        if (!std::isfinite(*e_idem)) return fail(BSM_ENONFINITE, "idempotency error is not finite");
        return BSM_OK;
    } catch (const Error &e) {
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}

extern "C" int lnv_forces(lnv_state *st, const bsm_matrix *dS, const bsm_matrix *dH, double *forces, double *mu_out)
{
    try {
        BSM_REQUIRE(st && dS && dH && forces, BSM_EINVAL, "NULL argument");
        Context *c = st->c;
        const bsm_pattern_s *PS = st->PS, *PH = st->PH, *PL = st->PL;
        BSM_REQUIRE(PS->cutoff == PH->cutoff && PS->nnzb == PH->nnzb, BSM_EPATTERN,
                    "forces need S and H on the same pattern");
        for (int k = 0; k < 3; ++k) {
            check_matrix(&dS[k], "dS");
            check_matrix(&dH[k], "dH");
            BSM_REQUIRE(dS[k].pattern == PS && dH[k].pattern == PH, BSM_EPATTERN,
                        "derivative blocks must be on the state's S and H patterns");
        }
        struct PrecGuard {   // FP64 products for the forces; the state's precision restored on every exit
            lnv_state_s *s;
            int p;
            ~PrecGuard() { s->prec = p; }
        } guard{st, st->prec};
        st->prec = BSM_F64;
        const int64_t ns = nelems(PS);
        Mat &X = st->X, &Y = st->Y, &W = st->W, &U = st->U;
        // chemical potential at the current L (canonical definition), as a step computes it
        st->mul_pair_sh(PL, st->L, X.p, X.d(), Y.d());               // X = L S, Y = L H
        st->mul_pair(X, Y, X, W, U);                                 // W = X X, U = Y X
        st->gradients();
        st->precondition(st->GE, st->PE);
        st->precondition(st->GN, st->PN);
        double gp[2];
        {
            const double *a[2] = {st->GN.d(), st->GN.d()}, *b[2] = {st->PN.d(), st->PE.d()};
            dots(c, 2, PL, a, b, gp);
        }
        const double mu = (st->prm.mode == LNV_CANONICAL && gp[0] > 0.0) ? gp[1] / gp[0] : st->mu;
        BSM_REQUIRE(std::isfinite(mu), BSM_ENONFINITE, "chemical potential is not finite");
        // K = 3 LSL - 2 LSLSL on P_S (exact: W L reaches r_L beyond P(r_L + r_S))
        Mat K(c, PS), K2(c, PS), Hp(c, PS), XM(c, PS), Wt(c, PS);
        st->mul(1.0, X.p, X.d(), PL, st->L, 0.0, PS, K.d());
        st->mul(1.0, W.p, W.d(), PL, st->L, 0.0, PS, K2.d());
        axpby(c, ns, -2.0, K2.d(), 3.0, K.d());
        // H' = H - mu S; M = (L H') L on P(r_L + r_S + r_S), exact where X M reads it
        axpby(c, ns, 1.0, st->H, 0.0, Hp.d());
        axpby(c, ns, -mu, st->S, 1.0, Hp.d());
        Mat &LH = st->XD;   // P_X scratch
        st->mul(1.0, PL, st->L, PS, Hp.d(), 0.0, LH.p, LH.d());
        const bsm_pattern_s *PM = derived_pattern_cached(PL, st->PX->cutoff + PS->cutoff);
        Mat M(c, PM);
        st->mul(1.0, LH.p, LH.d(), PL, st->L, 0.0, PM, M.d());
        st->mul(1.0, X.p, X.d(), PM, M.d(), 0.0, PS, XM.d());
        // Wt = Q - mu K with Q = 3 mask_S(M) - 2 (X M + (X M)^T)
        mask_copy(c, PM, M.d(), PS, Wt.d());
        add_transpose(c, PS, -2.0, XM.d(), 3.0, Wt.d());
        axpby(c, ns, -mu, K.d(), 1.0, Wt.d());
        DevBuf out(c, sizeof(double) * 3 * (size_t)PS->natoms);
        k_row_forces<<<PS->natoms, kForceThreads, 0, c->stream>>>(
            PS->b, PS->rowptr.as<int>(), PS->cols.as<int>(), K.d(), Wt.d(), (const double *)dH[0].blocks,
            (const double *)dH[1].blocks, (const double *)dH[2].blocks, (const double *)dS[0].blocks,
            (const double *)dS[1].blocks, (const double *)dS[2].blocks, out.as<double>());
        BSM_HIP_TRY(hipGetLastError());
        BSM_HIP_TRY(hipMemcpyAsync(forces, out.ptr, sizeof(double) * 3 * PS->natoms, hipMemcpyDeviceToHost,
                                   c->stream));
        BSM_HIP_TRY(hipStreamSynchronize(c->stream));
        if (mu_out) *mu_out = mu;
        for (int64_t e = 0; e < 3 * (int64_t)PS->natoms; ++e)
            if (!std::isfinite(forces[e])) return fail(BSM_ENONFINITE, "forces are not finite");
        return BSM_OK;
    } catch (const Error &e) {
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}

extern "C" int lnv_solve(lnv_state *st, const lnv_schedule *sch, lnv_solve_result *out)
{
    try {
        BSM_REQUIRE(st && sch && out, BSM_EINVAL, "NULL argument");
        BSM_REQUIRE(sch->n_stages >= 1 && sch->n_stages <= LNV_MAX_STAGES, BSM_EINVAL, "1..4 stages");
        *out = lnv_solve_result{};
        for (int s = 0; s < sch->n_stages; ++s) {
            const int p = sch->precision[s];
            BSM_REQUIRE(p == BSM_F64 || p == BSM_F32 || p == BSM_BF16, BSM_EINVAL, "bad stage precision");
            BSM_REQUIRE(sch->max_iter[s] >= 0, BSM_EINVAL, "bad stage max_iter");
            if (s > 0) {   // keep L, restart the conjugate gradients in the new precision
                lnv_params prm = st->prm;
                prm.init_from_z = 0;
                prm.product_precision = p;
                st->reset(prm);
            } else {
                st->prm.product_precision = p;
                st->prec = p;
            }
            bool stop = false;
            int it = 0;
            for (; it < sch->max_iter[s] && !stop; ++it) {
                lnv_result r{};
                const int code = st->step(&r);
                out->product_flops += r.product_flops;
                out->E = r.E;
                out->N = r.N;
                out->mu = r.mu;
                if (code != BSM_OK) {
                    out->status = code;
                    out->iterations[s] = it + 1;
                    return code;
                }
                if (st->n > 1) {
                    if (sch->tol_E[s] > 0 && std::fabs(r.dE) < sch->tol_E[s]) stop = true;
                    if (sch->stop_on_rise[s] && !(r.dE < 0.0)) stop = true;
                }
            }
            out->iterations[s] = it;
            if (s == sch->n_stages - 1) out->converged = (stop || sch->tol_E[s] <= 0) ? 1 : 0;
        }
        out->status = BSM_OK;
        return BSM_OK;
    } catch (const Error &e) {
        if (out) out->status = e.code;
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}
