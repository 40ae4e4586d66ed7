// Many independent products in one persistent launch, with a tile schedule
// chosen by measurement.
//
// A batch holds up to thousands of truncated products (C_p <- alpha_p
// mask(A_p B_p) + beta_p C_p), typically from independent systems of uneven
// size and orbital count (b = 4 or 9).  Every product keeps its own plan; the
// batch concatenates their tiles into one work list.  A fixed grid of
// one-wave workgroups stays resident and takes tiles from work queues by an
// atomic counter until the list is exhausted (every wave reaches the exit
// test).  A tile runs the same device code as in the separate launches (the
// LDS-ring tile for b = 9, the register-pipelined tiles for b = 4), in the
// workgroup's own LDS ring.
// Tiles write disjoint outputs, so the result does not depend on which wave
// takes which tile: it equals the separate products bit for bit.
//
// Schedule knobs, measured by bsm_batch_tune: the order of the work list (by
// product, heaviest tile first, or products interleaved), the resident waves
// per CU, and one global queue or one queue per XCD (each XCD then works
// through a contiguous, equally weighted slice of the list).
#include "bsm_internal.h"
#include "tiles.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <type_traits>
#include <vector>

namespace bsm {

// product kinds handled by the persistent kernel
enum { kKindF64Ring9 = 0, kKindF64Ring4 = 1, kKindF32Ring9 = 2, kKindF32Ring4 = 3 };
constexpr int kBatchRing = 2;   // LDS ring depth of the tiles
constexpr int kBatchRows = 8;   // rows per tile (the separate launches' default for b = 4 and 9)

struct BatchDesc {
    int kind;
    int pad;
    unsigned a_bytes, b_bytes;   // operand sizes (buffer copies)
    const int *hdr;
    const int64_t *ebeg;
    const int *ent;
    const void *A;
    const void *B;
    double *C;
    double alpha, beta;
};

namespace {

constexpr int kCUs = 256;

__global__ void k_zero_counters(int n, unsigned *c)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}

// One kernel per batch precision (F64 = true: FP64 operands; false: FP32) and
// per tile kind: KB = 9 or 4 runs only the b = 9 or b = 4 tiles (a work list of
// one orbital count, compiled with the registers and LDS that tile alone
// needs), KB = 0 either (mixed lists).  BUF: every product's operands fit
// buffer resources (a_bytes, b_bytes), and the tiles copy through them.
template <bool F64, bool BUF, int KB>
__global__ __launch_bounds__(64) void k_product_batch(const BatchDesc *__restrict__ desc, const int2 *__restrict__ items,
                                                      const int64_t *__restrict__ qbeg, int nq,
                                                      unsigned *__restrict__ counters, const double *__restrict__ zblk)
{
    using T = typename std::conditional<F64, double, float>::type;
    constexpr int kBytes9 = KB == 4 ? 0 : RingEntry<9, kBatchRows, T>::kBytes;
    constexpr int kBytes4 = KB == 9 ? 0 : RingEntry<4, kBatchRows, T>::kBytes;
    constexpr int kEntryBytes = kBytes9 > kBytes4 ? kBytes9 : kBytes4;
    __shared__ __attribute__((aligned(16))) char ring[kBatchRing * kEntryBytes];
    const int lane = threadIdx.x & 63;
    const int q = (int)(blockIdx.x % (unsigned)nq);   // workgroups are dealt round-robin to the XCDs
    const int64_t base = qbeg[q];
    const int64_t len = qbeg[q + 1] - base;
    while (true) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(&counters[q], 1u);
        t = (unsigned)__builtin_amdgcn_readfirstlane((int)__shfl((int)t, 0, 64));
        if ((int64_t)t >= len) break;
        const int2 it = items[base + t];
        const int p = __builtin_amdgcn_readfirstlane(it.x);
        const BatchDesc d = desc[p];
        const int kind = __builtin_amdgcn_readfirstlane(d.kind);
        if constexpr (F64) {
            if (KB == 9 || (KB == 0 && kind == kKindF64Ring9)) {
                if constexpr (KB != 4)
                    tile_ring<9, kBatchRows, kBatchRing, double, BUF>(it.y, d.hdr, d.ebeg, d.ent, (const double *)d.A,
                                                                 (const double *)d.B, zblk, d.C, d.alpha, d.beta,
                                                                 (lds_char_t *)ring, d.a_bytes, d.b_bytes);
            } else {
                if constexpr (KB != 9)
                    tile_ring<4, kBatchRows, kBatchRing, double, BUF>(it.y, d.hdr, d.ebeg, d.ent, (const double *)d.A,
                                                                 (const double *)d.B, zblk, d.C, d.alpha, d.beta,
                                                                 (lds_char_t *)ring, d.a_bytes, d.b_bytes);
            }
        } else {
            if (KB == 9 || (KB == 0 && kind == kKindF32Ring9)) {
                if constexpr (KB != 4)
                    tile_ring<9, kBatchRows, kBatchRing, float, BUF>(it.y, d.hdr, d.ebeg, d.ent, (const float *)d.A,
                                                                (const float *)d.B, (const float *)zblk, d.C, d.alpha,
                                                                d.beta, (lds_char_t *)ring, d.a_bytes, d.b_bytes);
            } else {
                if constexpr (KB != 9)
                    tile_ring<4, kBatchRows, kBatchRing, float, BUF>(it.y, d.hdr, d.ebeg, d.ent, (const float *)d.A,
                                                                (const float *)d.B, (const float *)zblk, d.C, d.alpha,
                                                                d.beta, (lds_char_t *)ring, d.a_bytes, d.b_bytes);
            }
        }
    }
}

__global__ void k_round_copy_b(int64_t n, const double *__restrict__ x, float *__restrict__ y, int bf16)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float f = (float)x[e];
    if (bf16) {
        unsigned u = __float_as_uint(f);
        if ((u & 0x7f800000u) == 0x7f800000u) {
            if (u & 0x007fffffu) u |= 0x00400000u;
            u &= 0xffff0000u;
        } else {
            u += 0x7fffu + ((u >> 16) & 1u);
            u &= 0xffff0000u;
        }
        f = __uint_as_float(u);
    }
    y[e] = f;
}

}  // namespace
}  // namespace bsm

using namespace bsm;

struct bsm_batch_s {
    Context *c = nullptr;
    int n = 0;
    int prec = BSM_F64;
    std::vector<Plan *> plans;
    std::vector<const bsm_pattern_s *> pa, pb, pc;
    std::vector<const double *> A, B;
    std::vector<double *> C;
    std::vector<int64_t> a_n, b_n;           // elements of each operand
    std::vector<DevBuf> a32, b32;           // rounded operand copies (FP32 / BF16 batches)
    std::vector<std::vector<int64_t>> work;  // entries per tile, per product
    std::vector<double> alpha, beta;
    DevBuf desc, items, qbeg, counters;
    double flops = 0.0;
    int64_t ntiles = 0;
    bool buf = true;          // every product's operands fit buffer resources
    bool tuned = false;
    bsm_batch_config best{};
    bsm_batch_config built{-1, -1, -1, -1};
    // work lists of the last schedule: one per launch (mode ONE_LAUNCH: all
    // products, kb = 0; mode PER_B: one per orbital count, kb = that count)
    struct Group {
        int kb;
        int64_t item0;   // first item of the group's list in `items`
    };
    std::vector<Group> groups;

    void build_schedule(const bsm_batch_config &cfg);
    void run(const bsm_batch_config &cfg);
};

void bsm_batch_s::build_schedule(const bsm_batch_config &cfg)
{
    if (cfg.mode == BSM_BATCH_SEPARATE) return;   // the products' own launches: no work list
    if (cfg.order == built.order && cfg.queues == built.queues && cfg.mode == built.mode) return;
    // each product's own launch order of its tiles (XCD-friendly interleaving of row groups)
    std::vector<std::vector<int>> order(n);
    for (int p = 0; p < n; ++p) {
        order[p].resize((size_t)plans[p]->ntiles);
        if (plans[p]->ntiles > 0)
            BSM_HIP_TRY(hipMemcpy(order[p].data(), plans[p]->order.ptr, sizeof(int) * (size_t)plans[p]->ntiles,
                                  hipMemcpyDeviceToHost));
    }
    std::vector<int2> all;         // every group's list, one after the other: (product, tile id)
    std::vector<int64_t> qb_all;   // per group, nq + 1 queue bounds (indices into the group's list)
    const int nq = std::max(1, cfg.queues);
    groups.clear();
    auto add_group = [&](int kb) {
        std::vector<int2> list;
        std::vector<int> ps;
        for (int p = 0; p < n; ++p)
            if (kb == 0 || plans[p]->b == kb) ps.push_back(p);
        if (ps.empty()) return;
        if (cfg.order == BSM_ORDER_BY_PRODUCT) {
            for (int p : ps)
                for (int64_t t = 0; t < plans[p]->ntiles; ++t) list.push_back(make_int2(p, order[p][t]));
        } else if (cfg.order == BSM_ORDER_INTERLEAVE) {
            int64_t longest = 0;
            for (int p : ps) longest = std::max(longest, plans[p]->ntiles);
            for (int64_t t = 0; t < longest; ++t)
                for (int p : ps)
                    if (t < plans[p]->ntiles) list.push_back(make_int2(p, order[p][t]));
        } else {   // heaviest tile first (longest-processing-time order for the dynamic queue)
            for (int p : ps)
                for (int64_t t = 0; t < plans[p]->ntiles; ++t) list.push_back(make_int2(p, order[p][t]));
            std::stable_sort(list.begin(), list.end(), [&](const int2 &x, const int2 &y) {
                const double wx = (double)work[x.x][x.y] * plans[x.x]->b * plans[x.x]->b;
                const double wy = (double)work[y.x][y.y] * plans[y.x]->b * plans[y.x]->b;
                return wx > wy;
            });
        }
        // queues: contiguous slices of the list with equal weight
        std::vector<int64_t> qb(nq + 1, 0);
        double total = 0.0;
        std::vector<double> w(list.size());
        for (size_t k = 0; k < list.size(); ++k) {
            w[k] = (double)(work[list[k].x][list[k].y] + 1) * plans[list[k].x]->b * plans[list[k].x]->b;
            total += w[k];
        }
        double acc = 0.0;
        int qi = 1;
        for (size_t k = 0; k < list.size() && qi < nq; ++k) {
            acc += w[k];
            while (qi < nq && acc >= total * qi / nq) qb[qi++] = (int64_t)k + 1;
        }
        while (qi < nq) qb[qi++] = (int64_t)list.size();
        qb[nq] = (int64_t)list.size();
        groups.push_back(Group{kb, (int64_t)all.size()});
        all.insert(all.end(), list.begin(), list.end());
        qb_all.insert(qb_all.end(), qb.begin(), qb.end());
    };
    if (cfg.mode == BSM_BATCH_PER_B) {
        add_group(9);
        add_group(4);
    } else {
        add_group(0);
    }
    items = DevBuf(c, sizeof(int2) * std::max<size_t>(1, all.size()));
    qbeg = DevBuf(c, sizeof(int64_t) * std::max<size_t>(1, qb_all.size()));
    if (!all.empty())
        BSM_HIP_TRY(hipMemcpyAsync(items.ptr, all.data(), sizeof(int2) * all.size(), hipMemcpyHostToDevice, c->stream));
    if (!qb_all.empty())
        BSM_HIP_TRY(hipMemcpyAsync(qbeg.ptr, qb_all.data(), sizeof(int64_t) * qb_all.size(), hipMemcpyHostToDevice,
                                   c->stream));
    BSM_HIP_TRY(hipStreamSynchronize(c->stream));
    built = cfg;
}

void bsm_batch_s::run(const bsm_batch_config &cfg)
{
    BSM_REQUIRE(cfg.mode >= BSM_BATCH_ONE_LAUNCH && cfg.mode <= BSM_BATCH_SEPARATE, BSM_EINVAL, "bad batch mode");
    if (cfg.mode == BSM_BATCH_SEPARATE) {
        // each product in its own launch, with the plan and kernel a single product call uses
        for (int p = 0; p < n; ++p)
            launch_product_mixed(c, get_plan(c, pa[p], pb[p], pc[p]), prec, alpha[p], pa[p], A[p], pb[p], B[p],
                                 beta[p], pc[p], C[p]);
        return;
    }
    BSM_REQUIRE(cfg.order >= 0 && cfg.order <= 2, BSM_EINVAL, "bad batch order");
    BSM_REQUIRE(cfg.waves_per_cu >= 4 && cfg.waves_per_cu <= 32 && cfg.waves_per_cu % 4 == 0, BSM_EINVAL,
                "waves per CU must be 4..32, a multiple of 4");
    BSM_REQUIRE(cfg.queues == 1 || cfg.queues == 8, BSM_EINVAL, "queues must be 1 or 8");
    build_schedule(cfg);
    hipStream_t st = c->stream;
    if (prec != BSM_F64) {
        for (int p = 0; p < n; ++p) {
            k_round_copy_b<<<(unsigned)((a_n[p] + 255) / 256), 256, 0, st>>>(a_n[p], A[p], a32[p].as<float>(),
                                                                             prec == BSM_BF16);
            k_round_copy_b<<<(unsigned)((b_n[p] + 255) / 256), 256, 0, st>>>(b_n[p], B[p], b32[p].as<float>(),
                                                                             prec == BSM_BF16);
        }
    }
    const int nq = cfg.queues;
    k_zero_counters<<<1, 64, 0, st>>>(nq * (int)groups.size(), counters.as<unsigned>());
    const int blocks = kCUs * cfg.waves_per_cu;   // one wave each
    for (size_t g = 0; g < groups.size(); ++g) {
        auto go = [&](auto kern) {
            kern<<<blocks, 64, 0, st>>>(desc.as<BatchDesc>(), items.as<int2>() + groups[g].item0,
                                        qbeg.as<int64_t>() + g * (nq + 1), nq, counters.as<unsigned>() + g * nq,
                                        c->zero_block.as<double>());
        };
#define BATCH_KERNELS(KB)                                                                          \
        if (prec == BSM_F64)                                                                       \
            buf ? go(k_product_batch<true, true, KB>) : go(k_product_batch<true, false, KB>);      \
        else                                                                                       \
            buf ? go(k_product_batch<false, true, KB>) : go(k_product_batch<false, false, KB>)
        if (groups[g].kb == 9) BATCH_KERNELS(9);
        else if (groups[g].kb == 4) BATCH_KERNELS(4);
        else BATCH_KERNELS(0);
#undef BATCH_KERNELS
        BSM_HIP_TRY(hipGetLastError());
    }
}

#define BATCH_BEGIN try {
#define BATCH_END                                                     \
    }                                                                 \
    catch (const Error &e) { return fail(e.code, e.msg); }            \
    catch (...) { return fail(BSM_EINVAL, "unknown error"); }

extern "C" {

int bsm_batch_create(bsm_ctx ctx, int n, const bsm_matrix *A, const bsm_matrix *B, const bsm_matrix *C,
                     const double *alpha, const double *beta, int precision, bsm_batch *out)
{
    BATCH_BEGIN
    BSM_REQUIRE(ctx && A && B && C && alpha && beta && out, BSM_EINVAL, "NULL argument");
    BSM_REQUIRE(n >= 1, BSM_EINVAL, "empty batch");
    BSM_REQUIRE(precision == BSM_F64 || precision == BSM_F32 || precision == BSM_BF16, BSM_EINVAL,
                "bad precision");
    std::unique_ptr<bsm_batch_s> bt(new bsm_batch_s());
    Context *c = &ctx->c;
    bt->c = c;
    bt->n = n;
    bt->prec = precision;
    std::vector<BatchDesc> d(n);
    for (int p = 0; p < n; ++p) {
        check_matrix(&A[p], "A");
        check_matrix(&B[p], "B");
        check_matrix(&C[p], "C");
        check_same_shape(&A[p], &B[p]);
        check_same_shape(&A[p], &C[p]);
        const int b = C[p].pattern->b;
        BSM_REQUIRE(b == 4 || b == 9, BSM_EINVAL, "batched products support b = 4 and 9");
        // LDS-ring tiles of 8 rows (the plans the separate launches use by default)
        Plan *plan = get_plan_kind(c, A[p].pattern, B[p].pattern, C[p].pattern, 4, kBatchRows);
        bt->plans.push_back(plan);
        bt->pa.push_back(A[p].pattern);
        bt->pb.push_back(B[p].pattern);
        bt->pc.push_back(C[p].pattern);
        bt->alpha.push_back(alpha[p]);
        bt->beta.push_back(beta[p]);
        bt->A.push_back((const double *)A[p].blocks);
        bt->B.push_back((const double *)B[p].blocks);
        bt->C.push_back((double *)C[p].blocks);
        bt->a_n.push_back(nelems(A[p].pattern));
        bt->b_n.push_back(nelems(B[p].pattern));
        bt->flops += plan->flops;
        bt->ntiles += plan->ntiles;
        // per-tile entry counts: the schedule's weights
        std::vector<int64_t> eb((size_t)plan->ntiles + 1);
        BSM_HIP_TRY(hipMemcpy(eb.data(), plan->ebeg.ptr, sizeof(int64_t) * eb.size(), hipMemcpyDeviceToHost));
        std::vector<int64_t> w((size_t)plan->ntiles);
        for (int64_t t = 0; t < plan->ntiles; ++t) w[t] = eb[t + 1] - eb[t];
        bt->work.push_back(std::move(w));
        BatchDesc &x = d[p];
        x.hdr = plan->hdr.as<int>();
        x.ebeg = plan->ebeg.as<int64_t>();
        x.ent = plan->ent.as<int>();
        x.C = (double *)C[p].blocks;
        x.alpha = alpha[p];
        x.beta = beta[p];
        if (precision == BSM_F64) {
            x.kind = b == 9 ? kKindF64Ring9 : kKindF64Ring4;
            x.A = A[p].blocks;
            x.B = B[p].blocks;
        } else {
            x.kind = b == 9 ? kKindF32Ring9 : kKindF32Ring4;
            bt->a32.emplace_back(c, sizeof(float) * (size_t)std::max<int64_t>(1, bt->a_n.back()));
            bt->b32.emplace_back(c, sizeof(float) * (size_t)std::max<int64_t>(1, bt->b_n.back()));
            x.A = bt->a32.back().ptr;
            x.B = bt->b32.back().ptr;
        }
        const int64_t esz = precision == BSM_F64 ? 8 : 4;
        const int64_t ab = esz * bt->a_n.back(), bb = esz * bt->b_n.back();
        if (ab > (int64_t)kBufMaxBytes || bb > (int64_t)kBufMaxBytes || (((uintptr_t)x.A | (uintptr_t)x.B) & 15))
            bt->buf = false;
        x.a_bytes = (unsigned)std::min<int64_t>(ab, kBufMaxBytes);
        x.b_bytes = (unsigned)std::min<int64_t>(bb, kBufMaxBytes);
    }
    bt->desc = DevBuf(c, sizeof(BatchDesc) * n);
    BSM_HIP_TRY(hipMemcpy(bt->desc.ptr, d.data(), sizeof(BatchDesc) * n, hipMemcpyHostToDevice));
    bt->counters = DevBuf(c, sizeof(unsigned) * 64);
    bt->best = bsm_batch_config{BSM_ORDER_HEAVY_FIRST, 8, 1, BSM_BATCH_ONE_LAUNCH};
    *out = bt.release();
    return BSM_OK;
    BATCH_END
}

int bsm_batch_run(bsm_batch bt, const bsm_batch_config *cfg)
{
    BATCH_BEGIN
    BSM_REQUIRE(bt != nullptr, BSM_EINVAL, "batch is NULL");
    bt->run(cfg ? *cfg : bt->best);
    return BSM_OK;
    BATCH_END
}

int bsm_batch_flops(bsm_batch bt, double *flops)
{
    BATCH_BEGIN
    BSM_REQUIRE(bt && flops, BSM_EINVAL, "NULL argument");
    *flops = bt->flops;
    return BSM_OK;
    BATCH_END
}

int bsm_batch_tune(bsm_batch bt, int reps, bsm_batch_config *best, double *best_ms)
{
    BATCH_BEGIN
    BSM_REQUIRE(bt != nullptr && reps >= 1, BSM_EINVAL, "bad argument");
    hipStream_t st = bt->c->stream;
    hipEvent_t e0, e1;
    BSM_HIP_TRY(hipEventCreate(&e0));
    BSM_HIP_TRY(hipEventCreate(&e1));
    double best_t = INFINITY;
    bsm_batch_config arg{};
    const int orders[3] = {BSM_ORDER_HEAVY_FIRST, BSM_ORDER_BY_PRODUCT, BSM_ORDER_INTERLEAVE};
    const int waves[3] = {4, 8, 16};
    const int queues[2] = {1, 8};
    std::vector<bsm_batch_config> cands;
    // the separate launches first: a persistent schedule is kept only when it is faster
    cands.push_back(bsm_batch_config{BSM_ORDER_BY_PRODUCT, 8, 1, BSM_BATCH_SEPARATE});
    bool mixed_b = false;
    for (int p = 1; p < bt->n; ++p) mixed_b |= bt->plans[p]->b != bt->plans[0]->b;
    for (int mode : {BSM_BATCH_ONE_LAUNCH, BSM_BATCH_PER_B}) {
        if (mode == BSM_BATCH_PER_B && !mixed_b && bt->plans[0]->b == 9) continue;   // same as one launch of KB 9
        for (int o : orders)
            for (int q : queues)
                for (int w : waves) cands.push_back(bsm_batch_config{o, w, q, mode});
    }
    bt->run(bt->best);   // one warm-up (operand pages, caches, plans) for all candidates
    for (const bsm_batch_config &cfg : cands) {
        bt->build_schedule(cfg);   // host work kept out of the timing
        bt->run(cfg);              // each candidate's own warm-up (its kernel's first launch)
        BSM_HIP_TRY(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) bt->run(cfg);
        BSM_HIP_TRY(hipEventRecord(e1, st));
        BSM_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        BSM_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms / reps < best_t) {
            best_t = ms / reps;
            arg = cfg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    bt->best = arg;
    bt->tuned = true;
    if (best) *best = arg;
    if (best_ms) *best_ms = best_t;
    return BSM_OK;
    BATCH_END
}

int bsm_batch_destroy(bsm_batch bt)
{
    if (bt) {
        (void)hipStreamSynchronize(bt->c->stream);
        delete bt;
    }
    return BSM_OK;
}

}  // extern "C"
