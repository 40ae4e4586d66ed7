// Pattern-local elementwise kernels: axpby, blockwise symmetrisation and
// transposition, masked copies between patterns, identity and block input.
// All are HBM-bound streams over the block arrays.
#include "bsm_internal.h"

namespace bsm {
namespace {

constexpr int kT = 256;

inline unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kT - 1) / kT); }

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y)
{
    int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= n) return;
    y[e] = (b == 0.0) ? a * x[e] : a * x[e] + b * y[e];
}

// z <- a x + b y + c z, one element per thread (x or y may be z).  Each element
// is fma(c, z, fma(a, x, b y)), written out so that the paired kernel below
// gives the same bits.
__global__ void k_axpbypcz(int64_t n, double a, const double *x, double b, const double *y, double c,
                           double *z)
{
    int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= n) return;
    const double v = fma(a, x[e], b * y[e]);
    z[e] = (c == 0.0) ? v : fma(c, z[e], v);
}

// The same for an even count of 16-byte aligned elements, two per thread
// (16-byte loads and stores).
__global__ void k_axpbypcz2(int64_t n2, double a, const double2 *x, double b, const double2 *y, double c,
                            double2 *z)
{
    int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= n2) return;
    const double2 xv = x[e], yv = y[e];
    double2 v = make_double2(fma(a, xv.x, b * yv.x), fma(a, xv.y, b * yv.y));
    if (c != 0.0) {
        const double2 zv = z[e];
        v = make_double2(fma(c, zv.x, v.x), fma(c, zv.y, v.y));
    }
    z[e] = v;
}

// In place (M_ij, M_ji) <- ((M_ij + M_ji^T)/2, its transpose).  The thread of
// element (p, q) of slot s with s < t (or s == t and p <= q) writes both partners.
__global__ void k_symmetrize(int64_t nnz, int b, const int *__restrict__ tmap, double *__restrict__ M)
{
    const int bb = b * b;
    int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= nnz * bb) return;
    const int64_t s = e / bb;
    const int r = (int)(e - s * bb), p = r / b, q = r - p * b;
    const int64_t t = tmap[s];
    if (t < s || (t == s && p > q)) return;
    double *x = M + s * bb + p * b + q;
    double *y = M + t * bb + q * b + p;
    const double v = 0.5 * (*x + *y);
    *x = v;
    *y = v;
}

// out[s] <- alpha (M[s] + M[t]^T) + beta out[s]
__global__ void k_add_transpose(int64_t nnz, int b, const int *__restrict__ tmap, double alpha,
                                const double *__restrict__ M, double beta, double *__restrict__ out)
{
    const int bb = b * b;
    int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= nnz * bb) return;
    const int64_t s = e / bb;
    const int r = (int)(e - s * bb), p = r / b, q = r - p * b;
    const int64_t t = tmap[s];
    const double v = alpha * (M[e] + M[t * bb + q * b + p]);
    out[e] = (beta == 0.0) ? v : v + beta * out[e];
}

__device__ inline int find_in_row(const int *__restrict__ rowptr, const int *__restrict__ cols, int i, int j)
{
    int lo = rowptr[i], hi = rowptr[i + 1], end = hi;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cols[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && cols[lo] == j) ? lo : -1;
}

// One workgroup per chunk of destination slots: look up the source slot, copy or zero.
__global__ __launch_bounds__(kT) void k_mask_copy(int64_t nnzd, int b, const int *__restrict__ rowsD,
                                                  const int *__restrict__ colsD, const int *__restrict__ rpS,
                                                  const int *__restrict__ colsS, const double *__restrict__ src,
                                                  double *__restrict__ dst)
{
    __shared__ int ss[kT];
    const int bb = b * b;
    const int64_t base = (int64_t)blockIdx.x * kT;
    const int nsl = (int)min((int64_t)kT, nnzd - base);
    if (threadIdx.x < nsl) {
        const int64_t s = base + threadIdx.x;
        ss[threadIdx.x] = find_in_row(rpS, colsS, rowsD[s], colsD[s]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nsl * bb; e += kT) {
        const int ls = e / bb, r = e - ls * bb;
        const int t = ss[ls];
        dst[(base + ls) * bb + r] = (t >= 0) ? src[(int64_t)t * bb + r] : 0.0;
    }
}

__global__ void k_set_identity(int n, int b, const int *__restrict__ diag, double alpha, double *__restrict__ M)
{
    int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= (int64_t)n * b) return;
    const int i = (int)(e / b), p = (int)(e - (int64_t)i * b);
    M[(int64_t)diag[i] * b * b + p * b + p] = alpha;
}

__global__ __launch_bounds__(kT) void k_fill_blocks(int64_t count, int b, const int *__restrict__ rows,
                                                    const int *__restrict__ cols, const double *__restrict__ blocks,
                                                    int natoms, const int *__restrict__ rp,
                                                    const int *__restrict__ pc, double *__restrict__ M,
                                                    int *__restrict__ bad)
{
    __shared__ int ss[kT];
    const int bb = b * b;
    const int64_t base = (int64_t)blockIdx.x * kT;
    const int nsl = (int)min((int64_t)kT, count - base);
    if (threadIdx.x < nsl) {
        const int64_t s = base + threadIdx.x;
        const int r = rows[s], c = cols[s];
        int t = -1;
        if (r >= 0 && r < natoms && c >= 0 && c < natoms) t = find_in_row(rp, pc, r, c);
        if (t < 0) atomicOr(bad, 1);
        ss[threadIdx.x] = t;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nsl * bb; e += kT) {
        const int ls = e / bb, r = e - ls * bb;
        const int t = ss[ls];
        if (t >= 0) M[(int64_t)t * bb + r] = blocks[(base + ls) * bb + r];
    }
}

}  // namespace

void axpby(Context *ctx, int64_t n, double alpha, const double *x, double beta, double *y)
{
    if (n <= 0) return;
    k_axpby<<<grid1(n), kT, 0, ctx->stream>>>(n, alpha, x, beta, y);
    BSM_HIP_TRY(hipGetLastError());
}

void axpbypcz(Context *ctx, int64_t n, double a, const double *x, double b, const double *y, double c,
              double *z)
{
    if (n <= 0) return;
    const bool paired = (n % 2 == 0) && ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y) |
                                          reinterpret_cast<uintptr_t>(z)) % 16 == 0);
    if (paired)
        k_axpbypcz2<<<grid1(n / 2), kT, 0, ctx->stream>>>(n / 2, a, reinterpret_cast<const double2 *>(x), b,
                                                          reinterpret_cast<const double2 *>(y), c,
                                                          reinterpret_cast<double2 *>(z));
    else
        k_axpbypcz<<<grid1(n), kT, 0, ctx->stream>>>(n, a, x, b, y, c, z);
    BSM_HIP_TRY(hipGetLastError());
}

void symmetrize(Context *ctx, const bsm_pattern_s *P, double *M)
{
    const int64_t n = nelems(P);
    if (n <= 0) return;
    k_symmetrize<<<grid1(n), kT, 0, ctx->stream>>>(P->nnzb, P->b, P->tmap.as<int>(), M);
    BSM_HIP_TRY(hipGetLastError());
}

void add_transpose(Context *ctx, const bsm_pattern_s *P, double alpha, const double *M, double beta, double *out)
{
    const int64_t n = nelems(P);
    if (n <= 0) return;
    k_add_transpose<<<grid1(n), kT, 0, ctx->stream>>>(P->nnzb, P->b, P->tmap.as<int>(), alpha, M, beta, out);
    BSM_HIP_TRY(hipGetLastError());
}

void mask_copy(Context *ctx, const bsm_pattern_s *Ps, const double *src, const bsm_pattern_s *Pd, double *dst)
{
    if (Pd->nnzb <= 0) return;
    k_mask_copy<<<(unsigned)((Pd->nnzb + kT - 1) / kT), kT, 0, ctx->stream>>>(
        Pd->nnzb, Pd->b, Pd->rowidx.as<int>(), Pd->cols.as<int>(), Ps->rowptr.as<int>(), Ps->cols.as<int>(), src,
        dst);
    BSM_HIP_TRY(hipGetLastError());
}

void set_identity(Context *ctx, const bsm_pattern_s *P, double alpha, double *M)
{
    BSM_HIP_TRY(hipMemsetAsync(M, 0, sizeof(double) * (size_t)nelems(P), ctx->stream));
    const int64_t n = (int64_t)P->natoms * P->b;
    k_set_identity<<<grid1(n), kT, 0, ctx->stream>>>(P->natoms, P->b, P->diag.as<int>(), alpha, M);
    BSM_HIP_TRY(hipGetLastError());
}

void fill_blocks(Context *ctx, const bsm_pattern_s *P, double *M, int64_t count, const int32_t *rows,
                 const int32_t *cols, const double *blocks)
{
    hipStream_t st = ctx->stream;
    BSM_HIP_TRY(hipMemsetAsync(M, 0, sizeof(double) * (size_t)nelems(P), st));
    int *bad = ctx->err_flag.as<int>();
    BSM_HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), st));
    if (count > 0) {
        k_fill_blocks<<<(unsigned)((count + kT - 1) / kT), kT, 0, st>>>(
            count, P->b, rows, cols, blocks, P->natoms, P->rowptr.as<int>(), P->cols.as<int>(), M, bad);
        BSM_HIP_TRY(hipGetLastError());
    }
    int h = 0;
    BSM_HIP_TRY(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    BSM_REQUIRE(h == 0, BSM_EPATTERN, "a block falls outside the matrix pattern");
}

}  // namespace bsm
