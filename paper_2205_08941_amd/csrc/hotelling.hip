// Hotelling / Schulz iteration for the truncated inverse of the overlap matrix.
//
// The paper singles out linear-scaling inversion of the overlap matrix S as
// key to an efficient linear-scaling solution (Development Priorities).  The
// iteration Z <- 2Z - Z S Z (Hotelling 1943; Schulz 1933) squares the residual
// I - Z S at every step; truncating Z to its cutoff pattern after each step
// keeps it O(N), at the price of a residual floor where the iteration stalls.
#include "bsm_internal.h"

#include <cmath>
#include <vector>

namespace bsm {
namespace {

// ||I - Z S||_F from T = Z S held exactly, summed elementwise over (T - I)^2
// (the equal form N_b - 2 Tr T + ||T||_F^2 cancels to ~1e-13 N_b in r^2).
double residual(Context *c, const bsm_pattern_s *PT, const double *T, double)
{
    const double r2 = dist_identity_sq(c, PT, T);
    if (!std::isfinite(r2)) return NAN;
    return std::sqrt(r2);
}

}  // namespace
}  // namespace bsm

using namespace bsm;

extern "C" int hotelling_inverse(bsm_ctx ctx, const bsm_matrix *S, const bsm_matrix *Z, const hot_params *prm,
                                 hot_result *res)
{
    try {
        BSM_REQUIRE(ctx && prm && res, BSM_EINVAL, "NULL argument");
        check_matrix(S, "S");
        check_matrix(Z, "Z");
        check_same_shape(S, Z);
        BSM_REQUIRE(prm->max_iter >= 0, BSM_EINVAL, "max_iter is negative");
        BSM_REQUIRE(S->blocks != Z->blocks, BSM_EINVAL, "S and Z alias");
        Context *c = &ctx->c;
        const bsm_pattern_s *PS = S->pattern, *PZ = Z->pattern;
        const double *Sd = (const double *)S->blocks;
        double *Zd = (double *)Z->blocks;
        const double nb = (double)PS->natoms * PS->b;
        const int64_t nz = nelems(PZ);

        const bsm_pattern_s *PT = derived_pattern_cached(PZ, PZ->cutoff + PS->cutoff);
        const int64_t nt = nelems(PT);
        DevBuf T(c, sizeof(double) * nt), Tn(c, sizeof(double) * nt), Zw(c, sizeof(double) * nz),
            M(c, sizeof(double) * nz);
        Plan *pZS = get_plan(c, PZ, PS, PT);
        Plan *pTZ = get_plan(c, PT, PZ, PZ);

        res->n_residuals = 0;
        res->iterations = 0;
        res->alpha = 0.0;
        res->product_flops = 0.0;
        auto record = [&](double r) {
            if (res->residuals && res->n_residuals < res->capacity) res->residuals[res->n_residuals] = r;
            res->n_residuals++;
        };

        BSM_REQUIRE(prm->init_given >= 0 && prm->init_given <= 2, BSM_EINVAL, "bad init_given");
        res->start = prm->init_given ? 1 : 0;
        auto plain_alpha = [&]() {
            const double rho = max_abs_row_sum(c, PS, Sd);
            BSM_REQUIRE(std::isfinite(rho) && rho > 0.0, BSM_ENONFINITE,
                        "overlap matrix has a non-finite or zero row sum");
            return 1.0 / rho;
        };
        // plain start Z0 = alpha I into Z; T = Z0 S; r = its residual
        auto start_plain = [&](double &r) {
            res->alpha = plain_alpha();
            set_identity(c, PZ, res->alpha, Zd);
            launch_product_f64(c, pZS, 1.0, PZ, Zd, PS, Sd, 0.0, PT, T.as<double>());
            res->product_flops += pZS->flops;
            r = residual(c, PT, T.as<double>(), nb);
            res->start = 0;
        };
        double r = 0.0;
        if (prm->init_given == 0) {
            start_plain(r);
        } else {
            if (prm->init_given == 2) {   // Z holds a correction: Z0 = alpha I + Z
                res->alpha = plain_alpha();
                set_identity(c, PZ, res->alpha, Zw.as<double>());
                axpby(c, nz, 1.0, Zw.as<double>(), 1.0, Zd);
            }
            launch_product_f64(c, pZS, 1.0, PZ, Zd, PS, Sd, 0.0, PT, T.as<double>());
            res->product_flops += pZS->flops;
            r = residual(c, PT, T.as<double>(), nb);
            if (prm->init_given == 2) {
                // residual of the plain start alpha I (held in Zw), computed aside in Tn
                launch_product_f64(c, pZS, 1.0, PZ, Zw.as<double>(), PS, Sd, 0.0, PT, Tn.as<double>());
                res->product_flops += pZS->flops;
                const double rp = residual(c, PT, Tn.as<double>(), nb);
                if (!(std::isfinite(r) && r < rp)) {
                    BSM_HIP_TRY(hipMemcpyAsync(Zd, Zw.ptr, sizeof(double) * nz, hipMemcpyDeviceToDevice, c->stream));
                    std::swap(T, Tn);
                    r = rp;
                    res->start = 0;
                }
            }
        }
        if (!std::isfinite(r)) {
            res->status = BSM_ENONFINITE;
            record(r);
            return fail(BSM_ENONFINITE, "Hotelling residual is not finite");
        }
        record(r);
        // Z' = sym(mask_Z(2 Z - T Z)) until the tolerance, max_iter, stagnation or divergence
        auto iterate = [&](double &rr, int &it) {
            while (true) {
                if (prm->tol > 0 && rr < prm->tol * std::sqrt(nb)) return (int)BSM_OK;
                if (it == prm->max_iter) return prm->tol > 0 ? (int)BSM_ENOTCONV : (int)BSM_OK;
                launch_product_f64(c, pTZ, 1.0, PT, T.as<double>(), PZ, Zd, 0.0, PZ, M.as<double>());
                axpbypcz(c, nz, 2.0, Zd, -1.0, M.as<double>(), 0.0, Zw.as<double>());
                symmetrize(c, PZ, Zw.as<double>());
                launch_product_f64(c, pZS, 1.0, PZ, Zw.as<double>(), PS, Sd, 0.0, PT, Tn.as<double>());
                res->product_flops += pTZ->flops + pZS->flops;
                const double rn = residual(c, PT, Tn.as<double>(), nb);
                if (!std::isfinite(rn)) return (int)BSM_ENONFINITE;
                if (rn >= 0.99 * rr)   // no real progress: keep the current Z; the truncation floor or divergence
                    return rr <= 0.1 * std::sqrt(nb) ? (int)BSM_OK : (int)BSM_EDIVERGED;
                BSM_HIP_TRY(hipMemcpyAsync(Zd, Zw.ptr, sizeof(double) * nz, hipMemcpyDeviceToDevice, c->stream));
                std::swap(T, Tn);
                rr = rn;
                ++it;
                record(rr);
            }
        };
        int it = 0;
        int status = iterate(r, it);
        if (prm->init_given == 2 && res->start == 1 && status != BSM_OK && status != BSM_ENOTCONV) {
            // the given start failed: rerun from the plain start
            start_plain(r);
            record(r);
            it = 0;
            status = std::isfinite(r) ? iterate(r, it) : (int)BSM_ENONFINITE;
        }
        BSM_HIP_TRY(hipStreamSynchronize(c->stream));
        res->iterations = it;
        res->status = status;
        if (status == BSM_ENOTCONV) {
            set_error("Hotelling reached max_iter before the tolerance");
            return BSM_OK;
        }
        if (status != BSM_OK)
            return fail(status, status == BSM_EDIVERGED ? "Hotelling diverged: S is not positive definite"
                                                        : "Hotelling residual is not finite");
        return BSM_OK;
    } catch (const Error &e) {
        if (res) res->status = e.code;
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}
