// Inverse square root of the overlap matrix by the coupled Newton-Schulz
// iteration, truncated like the Hotelling inverse.
//
// The paper names linear-scaling inversion of the overlap matrix S as key
// (Development Priorities); S^-1/2, which symmetric (Loewdin)
// orthogonalisation needs, follows from the coupled iteration analysed by
// Higham (1997): with A = S / rho (rho the Gershgorin bound, so the spectrum
// of an SPD A lies in (0, 1]), Y0 = mask_Z(A) and Z0 = I,
//     P = Z Y,  T = (3 I - P) / 2,  Y <- Y T,  Z <- T Z
// converge to Y = A^1/2 and Z = A^-1/2, quadratically in I - Z Y.  Only the
// iterates are truncated (to Z's pattern, then symmetrised blockwise); P and T
// are held exactly on P(2 r_Z).
#include "bsm_internal.h"

#include <cmath>

using namespace bsm;

extern "C" int bsm_inverse_sqrt(bsm_ctx ctx, const bsm_matrix *S, const bsm_matrix *Z, const bsm_matrix *Y,
                                const hot_params *prm, hot_result *res)
{
    try {
        BSM_REQUIRE(ctx && prm && res, BSM_EINVAL, "NULL argument");
        check_matrix(S, "S");
        check_matrix(Z, "Z");
        check_same_shape(S, Z);
        if (Y) {
            check_matrix(Y, "Y");
            BSM_REQUIRE(Y->pattern == Z->pattern, BSM_EPATTERN, "Y must be on Z's pattern");
            BSM_REQUIRE(Y->blocks != Z->blocks && Y->blocks != S->blocks, BSM_EINVAL, "Y aliases S or Z");
        }
        BSM_REQUIRE(prm->max_iter >= 0, BSM_EINVAL, "max_iter is negative");
        BSM_REQUIRE(prm->init_given == 0, BSM_EINVAL, "the inverse square root starts from S / rho (init_given 0)");
        BSM_REQUIRE(S->blocks != Z->blocks, BSM_EINVAL, "S and Z alias");
        Context *c = &ctx->c;
        const bsm_pattern_s *PS = S->pattern, *PZ = Z->pattern;
        const double *Sd = (const double *)S->blocks;
        const double nb = (double)PS->natoms * PS->b;
        const int64_t nz = nelems(PZ);
        const bsm_pattern_s *P2 = derived_pattern_cached(PZ, 2.0 * PZ->cutoff);
        const int64_t n2 = nelems(P2);
        DevBuf Yi(c, sizeof(double) * nz), Yn(c, sizeof(double) * nz), Zi(c, sizeof(double) * nz),
            Zn(c, sizeof(double) * nz), P(c, sizeof(double) * n2), Pn(c, sizeof(double) * n2),
            T(c, sizeof(double) * n2);
        Plan *pZY = get_plan(c, PZ, PZ, P2);   // P = Z Y
        Plan *pYT = get_plan(c, PZ, P2, PZ);   // Y T
        Plan *pTZ = get_plan(c, P2, PZ, PZ);   // T Z

        res->n_residuals = 0;
        res->iterations = 0;
        res->product_flops = 0.0;
        res->start = 0;
        auto record = [&](double r) {
            if (res->residuals && res->n_residuals < res->capacity) res->residuals[res->n_residuals] = r;
            res->n_residuals++;
        };
        // ||I - X||_F over P(2 r_Z), summed elementwise (deterministic)
        auto residual = [&](const double *X) {
            const double r2 = dist_identity_sq(c, P2, X);
            return std::isfinite(r2) ? std::sqrt(r2) : NAN;
        };

        const double rho = max_abs_row_sum(c, PS, Sd);
        BSM_REQUIRE(std::isfinite(rho) && rho > 0.0, BSM_ENONFINITE, "overlap matrix has a non-finite or zero row sum");
        res->alpha = 1.0 / rho;
        mask_copy(c, PS, Sd, PZ, Yi.as<double>());                    // Y0 = mask_Z(S) / rho
        axpby(c, nz, res->alpha, Yi.as<double>(), 0.0, Yi.as<double>());
        set_identity(c, PZ, 1.0, Zi.as<double>());                     // Z0 = I
        launch_product_f64(c, pZY, 1.0, PZ, Zi.as<double>(), PZ, Yi.as<double>(), 0.0, P2, P.as<double>());
        res->product_flops += pZY->flops;
        double r = residual(P.as<double>());
        record(r);
        int status = std::isfinite(r) ? (int)BSM_OK : (int)BSM_ENONFINITE;
        int it = 0;
        while (status == BSM_OK) {
            if (prm->tol > 0 && r < prm->tol * std::sqrt(nb)) break;
            if (it == prm->max_iter) {
                status = prm->tol > 0 ? (int)BSM_ENOTCONV : (int)BSM_OK;
                break;
            }
            set_identity(c, P2, 1.5, T.as<double>());                  // T = 3/2 I - P / 2
            axpby(c, n2, -0.5, P.as<double>(), 1.0, T.as<double>());
            launch_product_f64(c, pYT, 1.0, PZ, Yi.as<double>(), P2, T.as<double>(), 0.0, PZ, Yn.as<double>());
            symmetrize(c, PZ, Yn.as<double>());
            launch_product_f64(c, pTZ, 1.0, P2, T.as<double>(), PZ, Zi.as<double>(), 0.0, PZ, Zn.as<double>());
            symmetrize(c, PZ, Zn.as<double>());
            launch_product_f64(c, pZY, 1.0, PZ, Zn.as<double>(), PZ, Yn.as<double>(), 0.0, P2, Pn.as<double>());
            res->product_flops += pYT->flops + pTZ->flops + pZY->flops;
            const double rn = residual(Pn.as<double>());
            if (!std::isfinite(rn)) {
                status = BSM_ENONFINITE;
                break;
            }
            if (rn >= 0.99 * r) {   // no real progress: keep the current iterates; the floor or divergence
                status = r <= 0.1 * std::sqrt(nb) ? (int)BSM_OK : (int)BSM_EDIVERGED;
                break;
            }
            std::swap(Yi, Yn);
            std::swap(Zi, Zn);
            std::swap(P, Pn);
            r = rn;
            ++it;
            record(r);
        }
        // S^-1/2 = Z / sqrt(rho), S^1/2 = sqrt(rho) Y
        axpby(c, nz, 1.0 / std::sqrt(rho), Zi.as<double>(), 0.0, (double *)Z->blocks);
        if (Y) axpby(c, nz, std::sqrt(rho), Yi.as<double>(), 0.0, (double *)Y->blocks);
        BSM_HIP_TRY(hipStreamSynchronize(c->stream));
        res->iterations = it;
        res->status = status;
        if (status == BSM_ENOTCONV) {
            set_error("inverse square root reached max_iter before the tolerance");
            return BSM_OK;
        }
        if (status != BSM_OK)
            return fail(status, status == BSM_EDIVERGED ? "inverse square root diverged: S is not positive definite"
                                                        : "inverse square root residual is not finite");
        return BSM_OK;
    } catch (const Error &e) {
        if (res) res->status = e.code;
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}
