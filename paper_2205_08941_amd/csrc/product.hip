// Truncated block-sparse products C <- alpha mask_{P_C}(A B) + beta C in FP64.
//
// The products of atom-block matrices cut back to a spatial-cutoff pattern are
// the operations the paper's linear-scaling solver is built from (Background
// and Current Status) and the part it already started to move to GPUs
// (Meeting the Exascale Challenges).
//
// Work decomposition (gfx950, wave64):
//   * a tile is one output row i and a run of JT consecutive blocks (i, j) of
//     that row of P_C; one wavefront owns one tile;
//   * lane l holds column c = l % b of output block j = l / b (JT = 64 / b
//     blocks per wave: 7 for b = 9, 16 for b = 4) and keeps that column's b
//     rows in registers for the whole contraction;
//   * the wave walks k over row i of A in ascending order (uniform), so the
//     b x b block A_ik has a wave-uniform address and is read through the
//     scalar cache into SGPRs, broadcast to every lane as an FMA operand;
//   * each lane walks column j of B (= row j of the symmetric pattern) with its
//     own merge pointer and takes part only when (k, j) is in P_B.  Only block
//     triples (i, k, j) that exist are multiplied: no zero fill, and the k-sum
//     of every output runs in ascending k (deterministic).
#include "bsm_internal.h"

namespace bsm {
namespace {

// Wave-uniform read-only view: loads through it become scalar loads when the
// address is uniform.
template <class T> using const_as4 = const __attribute__((address_space(4))) T;

template <int B> struct Tile {
    static constexpr int JT = 64 / B;
};

template <int B>
__global__ __launch_bounds__(256) void k_product_f64(
    const int2 *__restrict__ tiles, int64_t ntiles,
    const int *__restrict__ rpA, const int *__restrict__ cA, const double *__restrict__ vA,
    const int *__restrict__ rpB, const int *__restrict__ cB, const int *__restrict__ tmB,
    const double *__restrict__ vB,
    const int *__restrict__ rpC, const int *__restrict__ cC, double *__restrict__ vC,
    double alpha, double beta)
{
    constexpr int JT = Tile<B>::JT;
    constexpr int BB = B * B;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (wave >= ntiles) return;
    const int lane = threadIdx.x & 63;
    const int2 t = tiles[wave];
    const int i = __builtin_amdgcn_readfirstlane(t.x);
    const int s0 = __builtin_amdgcn_readfirstlane(t.y);
    const int send = rpC[i + 1];
    const int jl = lane / B, c = lane - jl * B;
    const int sC = s0 + jl;
    const bool valid = (jl < JT) && (sC < send);
    int p = 0, pend = 0;
    if (valid) {
        const int j = cC[sC];
        p = rpB[j];
        pend = rpB[j + 1];
    }
    double acc[B];
#pragma unroll
    for (int r = 0; r < B; ++r) acc[r] = 0.0;

    const int a0 = __builtin_amdgcn_readfirstlane(rpA[i]);
    const int a1 = __builtin_amdgcn_readfirstlane(rpA[i + 1]);
    const_as4<int> *cAu = (const_as4<int> *)cA;
    const_as4<double> *vAu = (const_as4<double> *)vA;
    for (int sa = a0; sa < a1; ++sa) {
        const int k = cAu[sa];
        while (p < pend && cB[p] < k) ++p;
        const bool act = (p < pend) && (cB[p] == k);
        if (__builtin_amdgcn_ballot_w64(act) == 0) continue;
        if (act) {
            const double *bp = vB + (int64_t)tmB[p] * BB + c;
            double bv[B];
#pragma unroll
            for (int m = 0; m < B; ++m) bv[m] = bp[m * B];
            const_as4<double> *ap = vAu + (int64_t)sa * BB;
#pragma unroll
            for (int r = 0; r < B; ++r) {
#pragma unroll
                for (int m = 0; m < B; ++m) acc[r] = fma(ap[r * B + m], bv[m], acc[r]);
            }
        }
    }
    if (valid) {
        double *cp = vC + (int64_t)sC * BB + c;
        if (beta == 0.0) {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * B] = alpha * acc[r];
        } else {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * B] = alpha * acc[r] + beta * cp[r * B];
        }
    }
}

// Same walk as the product, counting the block triples each lane takes part in.
template <int B>
__global__ __launch_bounds__(256) void k_count_triples(
    const int2 *__restrict__ tiles, int64_t ntiles, const int *__restrict__ rpA,
    const int *__restrict__ cA, const int *__restrict__ rpB, const int *__restrict__ cB,
    const int *__restrict__ rpC, const int *__restrict__ cC, unsigned long long *__restrict__ total)
{
    constexpr int JT = Tile<B>::JT;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (wave >= ntiles) return;
    const int lane = threadIdx.x & 63;
    const int2 t = tiles[wave];
    const int i = t.x, s0 = t.y;
    const int jl = lane / B, c = lane - jl * B;
    const int sC = s0 + jl;
    const bool valid = (jl < JT) && (sC < rpC[i + 1]) && (c == 0);
    long long cnt = 0;
    if (valid) {
        const int j = cC[sC];
        int p = rpB[j], pend = rpB[j + 1];
        for (int sa = rpA[i]; sa < rpA[i + 1]; ++sa) {
            const int k = cA[sa];
            while (p < pend && cB[p] < k) ++p;
            if (p < pend && cB[p] == k) ++cnt;
        }
    }
    // integer sums are exact, so the atomic order does not matter
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
    if (lane == 0 && cnt) atomicAdd(total, (unsigned long long)cnt);
}

__global__ void k_tiles_per_row(int n, int jt, const int *__restrict__ rp, int *__restrict__ cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cnt[i] = (rp[i + 1] - rp[i] + jt - 1) / jt;
}

__global__ void k_fill_tiles(int n, int jt, const int *__restrict__ rp, const int64_t *__restrict__ off,
                             int2 *__restrict__ tiles)
{
    int i = blockIdx.x;
    if (i >= n) return;
    int lo = rp[i], len = rp[i + 1] - lo;
    int nt = (len + jt - 1) / jt;
    for (int q = threadIdx.x; q < nt; q += blockDim.x) tiles[off[i] + q] = make_int2(i, lo + q * jt);
}

__global__ __launch_bounds__(1024) void k_scan64(int n, const int *__restrict__ in, int64_t *__restrict__ out)
{
    __shared__ long long part[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    const int chunk = (n + nt - 1) / nt;
    const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
    long long s = 0;
    for (int k = lo; k < hi; ++k) s += in[k];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        long long v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long run = part[t] - s;
    for (int k = lo; k < hi; ++k) {
        out[k] = run;
        run += in[k];
    }
    if (t == nt - 1) out[n] = part[t];
}

int jt_for(int b) { return 64 / b; }

template <int B>
void launch_b(hipStream_t st, const Plan *plan, double alpha, const bsm_pattern_s *PA, const double *A,
              const bsm_pattern_s *PB, const double *Bm, double beta, const bsm_pattern_s *PC, double *C)
{
    const int64_t waves = plan->ntiles;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    k_product_f64<B><<<grid, 256, 0, st>>>(
        plan->tiles.as<int2>(), waves, PA->rowptr.as<int>(), PA->cols.as<int>(), A,
        PB->rowptr.as<int>(), PB->cols.as<int>(), PB->tmap.as<int>(), Bm,
        PC->rowptr.as<int>(), PC->cols.as<int>(), C, alpha, beta);
}

template <int B>
void count_b(hipStream_t st, const Plan *plan, const bsm_pattern_s *PA, const bsm_pattern_s *PB,
             const bsm_pattern_s *PC, unsigned long long *total)
{
    const unsigned grid = (unsigned)((plan->ntiles + 3) / 4);
    k_count_triples<B><<<grid, 256, 0, st>>>(plan->tiles.as<int2>(), plan->ntiles, PA->rowptr.as<int>(),
                                             PA->cols.as<int>(), PB->rowptr.as<int>(), PB->cols.as<int>(),
                                             PC->rowptr.as<int>(), PC->cols.as<int>(), total);
}

#define BSM_FOR_EACH_B(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

}  // namespace

void build_tiles(Context *ctx, const bsm_pattern_s *PC, Plan *plan)
{
    hipStream_t st = ctx->stream;
    const int n = PC->natoms;
    plan->jt = jt_for(PC->b);
    DevBuf cnt(ctx, sizeof(int) * n), off(ctx, sizeof(int64_t) * (n + 1));
    k_tiles_per_row<<<(n + 255) / 256, 256, 0, st>>>(n, plan->jt, PC->rowptr.as<int>(), cnt.as<int>());
    k_scan64<<<1, 1024, 0, st>>>(n, cnt.as<int>(), off.as<int64_t>());
    int64_t total = 0;
    BSM_HIP_TRY(hipMemcpyAsync(&total, off.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    plan->ntiles = total;
    plan->tiles = DevBuf(ctx, sizeof(int2) * (size_t)std::max<int64_t>(total, 1));
    k_fill_tiles<<<n, 64, 0, st>>>(n, plan->jt, PC->rowptr.as<int>(), off.as<int64_t>(),
                                   plan->tiles.as<int2>());
    BSM_HIP_TRY(hipGetLastError());
}

int64_t count_triples(Context *ctx, const bsm_pattern_s *PA, const bsm_pattern_s *PB,
                      const bsm_pattern_s *PC, const Plan *plan)
{
    hipStream_t st = ctx->stream;
    DevBuf total(ctx, sizeof(unsigned long long));
    BSM_HIP_TRY(hipMemsetAsync(total.ptr, 0, sizeof(unsigned long long), st));
    if (plan->ntiles > 0) {
        switch (PC->b) {
#define X(b) \
    case b: count_b<b>(st, plan, PA, PB, PC, total.as<unsigned long long>()); break;
            BSM_FOR_EACH_B(X)
#undef X
            default: throw Error{BSM_EINVAL, "b must be in 1..16"};
        }
    }
    unsigned long long h = 0;
    BSM_HIP_TRY(hipMemcpyAsync(&h, total.ptr, sizeof(h), hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    return (int64_t)h;
}

void launch_product_f64(Context *ctx, const Plan *plan, double alpha, const bsm_pattern_s *PA,
                        const double *A, const bsm_pattern_s *PB, const double *Bm, double beta,
                        const bsm_pattern_s *PC, double *C)
{
    if (plan->ntiles == 0) return;
    hipStream_t st = ctx->stream;
    Context::ProfRec rec{plan, nullptr, nullptr};
    if (ctx->profiling) {
        rec.start = ctx->take_event();
        rec.stop = ctx->take_event();
        BSM_HIP_TRY(hipEventRecord(rec.start, st));
    }
    switch (PC->b) {
#define X(b) \
    case b: launch_b<b>(st, plan, alpha, PA, A, PB, Bm, beta, PC, C); break;
        BSM_FOR_EACH_B(X)
#undef X
        default: throw Error{BSM_EINVAL, "b must be in 1..16"};
    }
    BSM_HIP_TRY(hipGetLastError());
    if (ctx->profiling) {
        BSM_HIP_TRY(hipEventRecord(rec.stop, st));
        ctx->prof.push_back(rec);
    }
}

Plan *get_plan(Context *ctx, const bsm_pattern_s *A, const bsm_pattern_s *B, const bsm_pattern_s *C)
{
    auto key = std::make_tuple(A->id, B->id, C->id);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) return it->second.get();
    std::unique_ptr<Plan> plan(new Plan());
    plan->ids[0] = A->id;
    plan->ids[1] = B->id;
    plan->ids[2] = C->id;
    plan->cutoffs[0] = A->cutoff;
    plan->cutoffs[1] = B->cutoff;
    plan->cutoffs[2] = C->cutoff;
    plan->natoms = C->natoms;
    plan->b = C->b;
    build_tiles(ctx, C, plan.get());
    plan->triples = count_triples(ctx, A, B, C, plan.get());
    plan->flops = 2.0 * (double)C->b * C->b * C->b * (double)plan->triples;
    Plan *raw = plan.get();
    ctx->plans[key] = std::move(plan);
    return raw;
}

}  // namespace bsm
