// Contraction of block matrices to a few support functions per atom.
//
// The paper names an on-site equivalent of multi-site support functions
// (MSSF) for PAO basis sets among its development priorities: each atom's
// b orbitals are replaced by bc < b support functions, linear combinations of
// that atom's own orbitals, which shrinks every block of S, H (and so of the
// density matrix) from b x b to bc x bc.  With coefficients C_i (b x bc) the
// contracted blocks are M'_ij = C_i^T M_ij C_j on the same atom-pair pattern.
// The kernel is HBM-bound (one b x b block in, one bc x bc block out).
#include "bsm_internal.h"

namespace bsm {
namespace {

constexpr int kThreads = 256;

// one thread per output element (slot, alpha, beta): sum_a C_i[a][alpha] sum_c M_ij[a][c] C_j[c][beta]
__global__ __launch_bounds__(kThreads) void k_contract(int64_t nnzb, int b, int bc, const int *__restrict__ rows,
                                                       const int *__restrict__ cols, const double *__restrict__ coef,
                                                       const double *__restrict__ M, double *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int bc2 = bc * bc;
    if (e >= nnzb * bc2) return;
    const int64_t s = e / bc2;
    const int r = (int)(e - s * bc2), al = r / bc, be = r - al * bc;
    const double *Ci = coef + (int64_t)rows[s] * b * bc, *Cj = coef + (int64_t)cols[s] * b * bc;
    const double *Mb = M + s * b * b;
    double acc = 0.0;
    for (int a = 0; a < b; ++a) {
        double t = 0.0;
        for (int c = 0; c < b; ++c) t += Mb[a * b + c] * Cj[c * bc + be];
        acc += Ci[a * bc + al] * t;
    }
    out[e] = acc;
}

}  // namespace
}  // namespace bsm

using namespace bsm;

extern "C" int bsm_contract(bsm_ctx ctx, const bsm_matrix *M, const double *coef, const bsm_matrix *out)
{
    try {
        BSM_REQUIRE(ctx && M && coef && out, BSM_EINVAL, "NULL argument");
        check_matrix(M, "M");
        check_matrix(out, "out");
        const bsm_pattern_s *P = M->pattern, *Q = out->pattern;
        BSM_REQUIRE(P->natoms == Q->natoms && P->nnzb == Q->nnzb && P->cutoff == Q->cutoff, BSM_EPATTERN,
                    "out must be on a pattern of the same atoms and cutoff");
        BSM_REQUIRE(Q->b <= P->b, BSM_EINVAL, "more support functions than orbitals");
        BSM_REQUIRE(M->blocks != out->blocks, BSM_EINVAL, "M and out alias");
        Context *c = &ctx->c;
        const int64_t n = Q->nnzb * Q->b * Q->b;
        if (n > 0) {
            k_contract<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, c->stream>>>(
                P->nnzb, P->b, Q->b, P->rowidx.as<int>(), P->cols.as<int>(), coef, (const double *)M->blocks,
                (double *)out->blocks);
            BSM_HIP_TRY(hipGetLastError());
        }
        return BSM_OK;
    } catch (const Error &e) {
        return fail(e.code, e.msg);
    } catch (...) {
        return fail(BSM_EINVAL, "unknown error");
    }
}
