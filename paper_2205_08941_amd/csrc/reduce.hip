// Deterministic FP64 reductions: traces of products, Frobenius inner products,
// traces and the largest absolute row sum.
//
// The energy, electron count and their line-search polynomials of the LNV
// solver, and the Hotelling residual, are all traces of products of sparse
// matrices; they are read back to the host as a handful of FP64 scalars.
//
// Every reduction runs on a grid fixed by the input size, each workgroup sums
// a fixed range in a fixed tree order, and a second one-workgroup pass adds the
// partial sums in workgroup order: the result is bitwise reproducible.
#include "bsm_internal.h"

#include <cmath>
#include <mutex>

namespace bsm {
namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 256;   // slots per chunk: one transpose lookup per thread

struct Ptrs {
    const double *p[kRedSlots];
};

template <int CNT>
__device__ inline void block_reduce_store(double (&acc)[CNT], int count, double *__restrict__ partials)
{
    __shared__ double red[kThreads / 64][kRedSlots];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int n = 0; n < count; ++n) {
        double v = acc[n];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[w][n] = v;
    }
    __syncthreads();
    if (threadIdx.x < count) {
        double v = 0.0;
        for (int q = 0; q < kThreads / 64; ++q) v += red[q][threadIdx.x];
        partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = v;
    }
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

// Tr(A_n B_n) = sum over slots s = (i,k) of A of sum_pq A_n[s][p][q] B_n[t][q][p],
// t = slot of (k, i) in B's pattern (-1: block absent, contributes zero).
// BC > 0: the block size as a compile-time constant (no integer divisions by a
// runtime value in the element loop); 0: b from the argument.
template <int CNT, int BC>
__global__ __launch_bounds__(kThreads) void k_trace_products(
    int count, int b_arg, int64_t nnzA, const int *__restrict__ colsA, const int *__restrict__ rowsA,
    const int *__restrict__ tmapA, int same_pattern, const int *__restrict__ rpB,
    const int *__restrict__ colsB, Ptrs A, Ptrs Bp, double *__restrict__ partials)
{
    __shared__ int tslot[kChunk];
    double acc[CNT];
#pragma unroll
    for (int n = 0; n < CNT; ++n) acc[n] = 0.0;
    const int b = BC > 0 ? BC : b_arg;
    const int bb = b * b;
    const int64_t nchunks = (nnzA + kChunk - 1) / kChunk;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t base = ch * kChunk;
        const int nsl = (int)min((int64_t)kChunk, nnzA - base);
        __syncthreads();
        if (threadIdx.x < nsl) {
            const int64_t s = base + threadIdx.x;
            tslot[threadIdx.x] = same_pattern ? tmapA[s] : find_in_row(rpB, colsB, colsA[s], rowsA[s]);
        }
        __syncthreads();
        const int nel = nsl * bb;
        for (int e = threadIdx.x; e < nel; e += kThreads) {
            const int ls = e / bb, r = e - ls * bb;
            const int p = r / b, q = r - p * b;
            const int t = tslot[ls];
            if (t < 0) continue;
            const int64_t ia = (base + ls) * bb + r;
            const int64_t ib = (int64_t)t * bb + q * b + p;
#pragma unroll
            for (int n = 0; n < CNT; ++n)
                if (n < count) acc[n] = fma(A.p[n][ia], Bp.p[n][ib], acc[n]);
        }
    }
    block_reduce_store<CNT>(acc, count, partials);
}

// Fixed sets of traces Tr(A_{ai[n]} B_{bi[n]}) over few distinct matrices on
// one pattern: each element of each distinct matrix is loaded once and used by
// every trace that needs it.  Per trace the terms are summed in the same order
// as k_trace_products, so the results are the same bits.
struct EnergyTraces {   // Tr XY, Tr WY, Tr XX, Tr WX from A = {X, W}, B = {Y, X}
    static constexpr int na = 2, nb = 2, count = 4;
    static constexpr int ai[count] = {0, 1, 0, 1}, bi[count] = {0, 0, 1, 1};
};
struct LineSearchTraces {   // A = {X_D, X, M1, W, Q}, B = {Y, Y_D, X_D, X}
    static constexpr int na = 5, nb = 4, count = 15;
    static constexpr int ai[count] = {0, 1, 0, 1, 0, 2, 3, 4, 2, 4, 2, 3, 4, 2, 4};
    static constexpr int bi[count] = {0, 1, 1, 2, 2, 0, 1, 0, 1, 1, 3, 2, 3, 2, 2};
};

template <class TS, int CNT, int BC>
__global__ __launch_bounds__(kThreads) void k_trace_set(int b_arg, int64_t nnz, const int *__restrict__ tmap,
                                                        Ptrs A, Ptrs Bp, double *__restrict__ partials)
{
    static_assert(TS::count <= CNT, "trace count");
    __shared__ int tslot[kChunk];
    double acc[CNT];
#pragma unroll
    for (int n = 0; n < CNT; ++n) acc[n] = 0.0;
    const int b = BC > 0 ? BC : b_arg;
    const int bb = b * b;
    const int64_t nchunks = (nnz + kChunk - 1) / kChunk;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t base = ch * kChunk;
        const int nsl = (int)min((int64_t)kChunk, nnz - base);
        __syncthreads();
        if (threadIdx.x < nsl) tslot[threadIdx.x] = tmap[base + threadIdx.x];
        __syncthreads();
        const int nel = nsl * bb;
        for (int e = threadIdx.x; e < nel; e += kThreads) {
            const int ls = e / bb, r = e - ls * bb;
            const int p = r / b, q = r - p * b;
            const int64_t ia = (base + ls) * bb + r;
            const int64_t ib = (int64_t)tslot[ls] * bb + q * b + p;
            double av[TS::na], bv[TS::nb];
#pragma unroll
            for (int j = 0; j < TS::na; ++j) av[j] = A.p[j][ia];
#pragma unroll
            for (int j = 0; j < TS::nb; ++j) bv[j] = Bp.p[j][ib];
#pragma unroll
            for (int n = 0; n < TS::count; ++n) acc[n] = fma(av[TS::ai[n]], bv[TS::bi[n]], acc[n]);
        }
    }
    block_reduce_store<CNT>(acc, TS::count, partials);
}

template <int CNT>
__global__ __launch_bounds__(kThreads) void k_dots(int count, int64_t nel, Ptrs A, Ptrs Bp,
                                                    double *__restrict__ partials)
{
    double acc[CNT];
#pragma unroll
    for (int n = 0; n < CNT; ++n) acc[n] = 0.0;
    const int64_t per = (nel + gridDim.x - 1) / gridDim.x;
    const int64_t lo = per * blockIdx.x, hi = min(nel, lo + per);
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
#pragma unroll
        for (int n = 0; n < CNT; ++n)
            if (n < count) acc[n] = fma(A.p[n][e], Bp.p[n][e], acc[n]);
    }
    block_reduce_store<CNT>(acc, count, partials);
}

__global__ __launch_bounds__(kThreads) void k_trace_single(int n, int b, const int *__restrict__ diag,
                                                           const double *__restrict__ A,
                                                           double *__restrict__ partials)
{
    double acc[1] = {0.0};
    const int per = (n + gridDim.x - 1) / gridDim.x;
    const int lo = per * blockIdx.x, hi = min(n, lo + per);
    for (int i = lo + threadIdx.x; i < hi; i += kThreads) {
        const double *d = A + (int64_t)diag[i] * b * b;
        double s = 0.0;
        for (int p = 0; p < b; ++p) s += d[p * b + p];
        acc[0] += s;
    }
    block_reduce_store<1>(acc, 1, partials);
}

// ||M - I||_F^2 summed elementwise (the identity sits on the diagonal slots).
__global__ __launch_bounds__(kThreads) void k_dist_identity(int64_t nnz, int b, const int *__restrict__ rows,
                                                            const int *__restrict__ cols,
                                                            const double *__restrict__ M,
                                                            double *__restrict__ partials)
{
    double acc[1] = {0.0};
    const int bb = b * b;
    const int64_t nel = nnz * bb;
    const int64_t per = (nel + gridDim.x - 1) / gridDim.x;
    const int64_t lo = per * blockIdx.x, hi = min(nel, lo + per);
    for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
        const int64_t s = e / bb;
        const int r = (int)(e - s * bb);
        const bool one = rows[s] == cols[s] && (r / b) == (r % b);
        const double v = M[e] - (one ? 1.0 : 0.0);
        acc[0] = fma(v, v, acc[0]);
    }
    block_reduce_store<1>(acc, 1, partials);
}

// Partial sums of every slot n added in workgroup order (one workgroup).
__device__ inline void k_finish_body(int count, int nparts, const double *__restrict__ partials,
                                     double *__restrict__ out)
{
    __shared__ double red[kThreads];
    for (int n = 0; n < count; ++n) {
        double v = 0.0;
        const int per = (nparts + kThreads - 1) / kThreads;
        const int lo = threadIdx.x * per, hi = min(nparts, lo + per);
        for (int q = lo; q < hi; ++q) v += partials[(size_t)n * nparts + q];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int off = kThreads / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[n] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_finish(int count, int nparts, const double *__restrict__ partials,
                                                     double *__restrict__ out)
{
    k_finish_body(count, nparts, partials, out);
}

// Largest absolute row sum (max over scalar rows of sum_j |A_ij|); max is
// order-independent, so an integer atomicMax on the non-negative bit pattern is exact.
__global__ void k_row_abs_max(int n, int b, const int *__restrict__ rowptr, const double *__restrict__ A,
                              unsigned long long *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * b) return;
    const int i = (int)(t / b), p = (int)(t - (int64_t)i * b);
    double s = 0.0;
    for (int sl = rowptr[i]; sl < rowptr[i + 1]; ++sl) {
        const double *blk = A + (int64_t)sl * b * b + p * b;
        for (int q = 0; q < b; ++q) s += fabs(blk[q]);
    }
    if (!(s >= 0.0)) s = __builtin_inf();   // NaN row: report as non-finite
    atomicMax(out, (unsigned long long)__double_as_longlong(s));
}

int grid_for(int64_t work)
{
    int64_t g = (work + kThreads - 1) / kThreads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, kRedBlocks));
}

void finish(Context *ctx, int count, int nparts, double *out)
{
    hipStream_t st = ctx->stream;
    double *dev_out = ctx->red_partials.as<double>() + (size_t)kRedSlots * kRedBlocks;
    k_finish<<<1, kThreads, 0, st>>>(count, nparts, ctx->red_partials.as<double>(), dev_out);
    BSM_HIP_TRY(hipGetLastError());
    BSM_HIP_TRY(hipMemcpyAsync(ctx->host_scalars, dev_out, sizeof(double) * count, hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    for (int n = 0; n < count; ++n) out[n] = ctx->host_scalars[n];
}

}  // namespace

// ---------------------------------------------------------------- allocation-free trace
// Scratch of bsm_trace_product_noalloc: the per-workgroup partial sums of one
// trace (at most kRedBlocks of them, whatever the input size), then the result
// slot the final pass writes before it is copied to the caller's pointer.
// Each GPU the library runs on holds its own copy until the process ends; host
// code reaches it only through the address taken by trace_scratch_setup.
constexpr int kTraceScratchDoubles = kRedBlocks + 8;
static __device__ __align__(256) double scratch[kTraceScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double *g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, once taken

// Result of the allocation-free trace: *out = partial sums' total (one workgroup,
// the same fixed order as the general final pass).
__global__ __launch_bounds__(kThreads) void k_finish_to(int nparts, const double *__restrict__ partials,
                                                        double *__restrict__ out)
{
    k_finish_body(1, nparts, partials, out);
}

void trace_products(Context *ctx, int count, const bsm_pattern_s *PA, const double *const *A,
                    const bsm_pattern_s *PB, const double *const *B, double *out)
{
    BSM_REQUIRE(count >= 1 && count <= kRedSlots, BSM_EINVAL, "bad trace count");
    Ptrs pa{}, pb{};
    for (int n = 0; n < count; ++n) {
        pa.p[n] = A[n];
        pb.p[n] = B[n];
    }
    const int64_t nchunks = (PA->nnzb + kChunk - 1) / kChunk;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nchunks, kRedBlocks));
    const int same = (PA == PB) ? 1 : 0;
    hipStream_t st = ctx->stream;
#define LAUNCH_B(C, BC)                                                                                 \
    k_trace_products<C, BC><<<grid, kThreads, 0, st>>>(count, PA->b, PA->nnzb, PA->cols.as<int>(),        \
                                                       PA->rowidx.as<int>(), PA->tmap.as<int>(), same,   \
                                                       PB->rowptr.as<int>(), PB->cols.as<int>(), pa, pb, \
                                                       ctx->red_partials.as<double>())
#define LAUNCH(C)                             \
    do {                                      \
        if (PA->b == 9) LAUNCH_B(C, 9);       \
        else if (PA->b == 4) LAUNCH_B(C, 4);  \
        else LAUNCH_B(C, 0);                  \
    } while (0)
    if (count == 1) LAUNCH(1);
    else if (count <= 4) LAUNCH(4);
    else LAUNCH(kRedSlots);
#undef LAUNCH
#undef LAUNCH_B
    BSM_HIP_TRY(hipGetLastError());
    finish(ctx, count, grid, out);
}

// Take the device address of `scratch` on `device` (current), once per device.
void trace_scratch_setup(int device)
{
    BSM_REQUIRE(device >= 0 && device < kMaxDevices, BSM_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return;
    void *ptr = nullptr;
    BSM_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    BSM_REQUIRE(ptr != nullptr, BSM_EHIP, "no device address for the trace scratch");
    g_scratch_ptr[device] = (double *)ptr;
}

// Tr(A B) into a device double, asynchronously on the context stream, with the
// partial sums in `scratch`: no allocation, no synchronisation.  Same kernels,
// grid and order as trace_products with one trace, so the same bits.
void trace_product_noalloc(Context *ctx, const bsm_pattern_s *PA, const double *A, const bsm_pattern_s *PB,
                           const double *B, double *out_dev)
{
    double *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) ptr = g_scratch_ptr[ctx->device];
    }
    BSM_REQUIRE(ptr != nullptr, BSM_EHIP, "trace scratch address not taken for this device");
    Ptrs pa{}, pb{};
    pa.p[0] = A;
    pb.p[0] = B;
    const int64_t nchunks = (PA->nnzb + kChunk - 1) / kChunk;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nchunks, kRedBlocks));
    static_assert(kRedBlocks <= kTraceScratchDoubles, "scratch holds every partial sum");
    const int same = (PA == PB) ? 1 : 0;
    hipStream_t st = ctx->stream;
#define LAUNCH_B(BC)                                                                                       \
    k_trace_products<1, BC><<<grid, kThreads, 0, st>>>(1, PA->b, PA->nnzb, PA->cols.as<int>(),           \
                                                       PA->rowidx.as<int>(), PA->tmap.as<int>(), same,   \
                                                       PB->rowptr.as<int>(), PB->cols.as<int>(), pa, pb, \
                                                       ptr)
    if (PA->b == 9) LAUNCH_B(9);
    else if (PA->b == 4) LAUNCH_B(4);
    else LAUNCH_B(0);
#undef LAUNCH_B
    BSM_HIP_TRY(hipGetLastError());
    k_finish_to<<<1, kThreads, 0, st>>>(grid, ptr, out_dev);
    BSM_HIP_TRY(hipGetLastError());
}

void trace_set(Context *ctx, int kind, const bsm_pattern_s *P, const double *const *A, const double *const *B,
               double *out)
{
    BSM_REQUIRE(kind == kTracesEnergy || kind == kTracesLineSearch, BSM_EINVAL, "bad trace set");
    Ptrs pa{}, pb{};
    const int na = kind == kTracesEnergy ? EnergyTraces::na : LineSearchTraces::na;
    const int nb = kind == kTracesEnergy ? EnergyTraces::nb : LineSearchTraces::nb;
    const int count = kind == kTracesEnergy ? EnergyTraces::count : LineSearchTraces::count;
    for (int j = 0; j < na; ++j) pa.p[j] = A[j];
    for (int j = 0; j < nb; ++j) pb.p[j] = B[j];
    const int64_t nchunks = (P->nnzb + kChunk - 1) / kChunk;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nchunks, kRedBlocks));
    hipStream_t st = ctx->stream;
    // the same accumulator widths as trace_products uses for these counts
    auto go = [&](auto ts, auto cnt) {
        using TS = decltype(ts);
        constexpr int C = decltype(cnt)::value;
        if (P->b == 9)
            k_trace_set<TS, C, 9><<<grid, kThreads, 0, st>>>(P->b, P->nnzb, P->tmap.as<int>(), pa, pb,
                                                              ctx->red_partials.as<double>());
        else if (P->b == 4)
            k_trace_set<TS, C, 4><<<grid, kThreads, 0, st>>>(P->b, P->nnzb, P->tmap.as<int>(), pa, pb,
                                                              ctx->red_partials.as<double>());
        else
            k_trace_set<TS, C, 0><<<grid, kThreads, 0, st>>>(P->b, P->nnzb, P->tmap.as<int>(), pa, pb,
                                                              ctx->red_partials.as<double>());
    };
    if (kind == kTracesEnergy) go(EnergyTraces{}, std::integral_constant<int, 4>{});
    else go(LineSearchTraces{}, std::integral_constant<int, kRedSlots>{});
    BSM_HIP_TRY(hipGetLastError());
    finish(ctx, count, grid, out);
}

void dots(Context *ctx, int count, const bsm_pattern_s *P, const double *const *A, const double *const *B,
          double *out)
{
    BSM_REQUIRE(count >= 1 && count <= kRedSlots, BSM_EINVAL, "bad dot count");
    Ptrs pa{}, pb{};
    for (int n = 0; n < count; ++n) {
        pa.p[n] = A[n];
        pb.p[n] = B[n];
    }
    const int64_t nel = nelems(P);
    const int grid = grid_for(nel);
    hipStream_t st = ctx->stream;
    if (count == 1) k_dots<1><<<grid, kThreads, 0, st>>>(count, nel, pa, pb, ctx->red_partials.as<double>());
    else if (count <= 4) k_dots<4><<<grid, kThreads, 0, st>>>(count, nel, pa, pb, ctx->red_partials.as<double>());
    else k_dots<kRedSlots><<<grid, kThreads, 0, st>>>(count, nel, pa, pb, ctx->red_partials.as<double>());
    BSM_HIP_TRY(hipGetLastError());
    finish(ctx, count, grid, out);
}

double trace_single(Context *ctx, const bsm_pattern_s *P, const double *A)
{
    const int grid = grid_for(P->natoms);
    k_trace_single<<<grid, kThreads, 0, ctx->stream>>>(P->natoms, P->b, P->diag.as<int>(), A,
                                                       ctx->red_partials.as<double>());
    BSM_HIP_TRY(hipGetLastError());
    double out = 0.0;
    finish(ctx, 1, grid, &out);
    return out;
}

double dist_identity_sq(Context *ctx, const bsm_pattern_s *P, const double *A)
{
    const int grid = grid_for(nelems(P));
    k_dist_identity<<<grid, kThreads, 0, ctx->stream>>>(P->nnzb, P->b, P->rowidx.as<int>(), P->cols.as<int>(), A,
                                                        ctx->red_partials.as<double>());
    BSM_HIP_TRY(hipGetLastError());
    double out = 0.0;
    finish(ctx, 1, grid, &out);
    return out;
}

double max_abs_row_sum(Context *ctx, const bsm_pattern_s *P, const double *A)
{
    hipStream_t st = ctx->stream;
    unsigned long long *dv = reinterpret_cast<unsigned long long *>(ctx->red_partials.as<double>() +
                                                                    (size_t)kRedSlots * kRedBlocks + kRedSlots);
    BSM_HIP_TRY(hipMemsetAsync(dv, 0, sizeof(unsigned long long), st));
    const int64_t rows = (int64_t)P->natoms * P->b;
    k_row_abs_max<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(P->natoms, P->b, P->rowptr.as<int>(), A, dv);
    BSM_HIP_TRY(hipGetLastError());
    BSM_HIP_TRY(hipMemcpyAsync(ctx->host_scalars, dv, sizeof(double), hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    return ctx->host_scalars[0];
}

}  // namespace bsm
