// C ABI entry points of libbsm: context, patterns, matrices, products, traces.
// Every entry point catches all exceptions and turns them into status codes.
#include "bsm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace bsm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

// ---------------------------------------------------------------- memory
void *Context::allocate(size_t bytes)
{
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (alloc_fn) {
        p = alloc_fn(bytes, user);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) p = nullptr;
    }
    if (!p) throw Error{BSM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    return p;
}

void Context::release(void *p)
{
    if (!p) return;
    if (free_fn) free_fn(p, user);
    else (void)hipFree(p);
}

float *Context::scratch_f32(int which, int64_t n)
{
    const size_t bytes = sizeof(float) * (size_t)std::max<int64_t>(n, 1);
    if (f32buf[which].bytes < bytes) {
        BSM_HIP_TRY(hipStreamSynchronize(stream));   // the old buffer may still be read
        f32buf[which] = DevBuf(this, bytes);
    }
    return f32buf[which].as<float>();
}

hipEvent_t Context::take_event()
{
    if (!event_pool.empty()) {
        hipEvent_t e = event_pool.back();
        event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    BSM_HIP_TRY(hipEventCreate(&e));
    return e;
}

void Context::clear_profile()
{
    for (auto &r : prof) {
        event_pool.push_back(r.start);
        event_pool.push_back(r.stop);
    }
    prof.clear();
}

void Context::retire_profile(const std::function<bool(const Plan *)> &pick)
{
    bool touched = false;
    for (auto &r : prof)
        if (pick(r.plan)) touched = true;
    if (touched) {
        (void)hipStreamSynchronize(stream);
        std::vector<ProfRec> keep;
        for (auto &r : prof) {
            if (pick(r.plan)) {
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, r.start, r.stop);
                auto &acc = retired[prof_key(r)];
                acc.launches += 1;
                acc.flops += r.plan->flops * r.products;
                acc.ms += ms;
                event_pool.push_back(r.start);
                event_pool.push_back(r.stop);
            } else {
                keep.push_back(r);
            }
        }
        prof.swap(keep);
    }
}

void Context::forget_pattern(uint64_t id)
{
    // recorded launches of plans about to be dropped are folded away first
    retire_profile([id](const Plan *p) { return p->ids[0] == id || p->ids[1] == id || p->ids[2] == id; });
    for (auto it = plans.begin(); it != plans.end();) {
        if (std::get<0>(it->first) == id || std::get<1>(it->first) == id || std::get<2>(it->first) == id)
            it = plans.erase(it);
        else
            ++it;
    }
}

DevBuf::DevBuf(Context *c, size_t n) : ctx(c), ptr(c->allocate(n)), bytes(n) {}

DevBuf::~DevBuf()
{
    if (ctx && ptr) ctx->release(ptr);
}

DevBuf &DevBuf::operator=(DevBuf &&o) noexcept
{
    if (this != &o) {
        if (ctx && ptr) ctx->release(ptr);
        ctx = o.ctx;
        ptr = o.ptr;
        bytes = o.bytes;
        o.ptr = nullptr;
        o.ctx = nullptr;
        o.bytes = 0;
    }
    return *this;
}

// ---------------------------------------------------------------- checks
int64_t nelems(const bsm_pattern_s *p) { return p->nnzb * (int64_t)p->b * p->b; }

void check_matrix(const bsm_matrix *M, const char *name)
{
    BSM_REQUIRE(M != nullptr, BSM_EINVAL, std::string(name) + " is NULL");
    BSM_REQUIRE(M->pattern != nullptr, BSM_EINVAL, std::string(name) + " has no pattern");
    BSM_REQUIRE(M->dtype == BSM_F64, BSM_EINVAL, std::string(name) + ": only BSM_F64 is supported here");
    BSM_REQUIRE(M->blocks != nullptr || M->pattern->nnzb == 0, BSM_EINVAL, std::string(name) + " blocks are NULL");
}

void check_same_shape(const bsm_matrix *A, const bsm_matrix *B)
{
    BSM_REQUIRE(A->pattern->natoms == B->pattern->natoms && A->pattern->b == B->pattern->b, BSM_EPATTERN,
                "atom count or orbitals per atom differ");
}

static bool overlaps(const bsm_matrix *X, const bsm_matrix *Y)
{
    const char *x0 = (const char *)X->blocks, *y0 = (const char *)Y->blocks;
    const char *x1 = x0 + sizeof(double) * nelems(X->pattern), *y1 = y0 + sizeof(double) * nelems(Y->pattern);
    return x0 < y1 && y0 < x1;
}

}  // namespace bsm

using namespace bsm;

#define BSM_API_BEGIN try {
#define BSM_API_END                                                  \
    }                                                                \
    catch (const bsm::Error &e) { return fail(e.code, e.msg); }      \
    catch (const std::bad_alloc &) { return fail(BSM_ENOMEM, "host allocation failed"); } \
    catch (const std::exception &e) { return fail(BSM_EINVAL, e.what()); } \
    catch (...) { return fail(BSM_EINVAL, "unknown error"); }

extern "C" {

const char *bsm_last_error(void) { return g_last_error.c_str(); }

int bsm_ctx_create(int device, void *hip_stream, bsm_alloc_fn alloc, bsm_free_fn free_fn, void *user,
                   bsm_ctx *out)
{
    BSM_API_BEGIN
    BSM_REQUIRE(out != nullptr, BSM_EINVAL, "out is NULL");
    BSM_REQUIRE((alloc == nullptr) == (free_fn == nullptr), BSM_EINVAL, "give both allocator callbacks or neither");
    int ndev = 0;
    BSM_HIP_TRY(hipGetDeviceCount(&ndev));
    BSM_REQUIRE(device >= 0 && device < ndev, BSM_EINVAL, "no such device");
    BSM_HIP_TRY(hipSetDevice(device));
    std::unique_ptr<bsm_ctx_s> c(new bsm_ctx_s());
    c->c.device = device;
    c->c.stream = (hipStream_t)hip_stream;
    c->c.alloc_fn = alloc;
    c->c.free_fn = free_fn;
    c->c.user = user;
    c->c.red_partials = DevBuf(&c->c, sizeof(double) * ((size_t)kRedSlots * kRedBlocks + kRedSlots + 8));
    c->c.err_flag = DevBuf(&c->c, 256);
    c->c.zero_block = DevBuf(&c->c, sizeof(double) * 256);
    BSM_HIP_TRY(hipMemset(c->c.zero_block.ptr, 0, sizeof(double) * 256));
    BSM_HIP_TRY(hipHostMalloc((void **)&c->c.host_scalars, sizeof(double) * 64, hipHostMallocDefault));
    trace_scratch_setup(device);   // the allocation-free trace's scratch on this device
    *out = c.release();
    return BSM_OK;
    BSM_API_END
}

int bsm_ctx_destroy(bsm_ctx ctx)
{
    BSM_API_BEGIN
    if (!ctx) return BSM_OK;
    (void)hipStreamSynchronize(ctx->c.stream);
    while (!ctx->c.derived.empty()) {
        bsm_pattern_s *d = ctx->c.derived.begin()->second;
        ctx->c.derived.erase(ctx->c.derived.begin());
        destroy_pattern(d);
    }
    ctx->c.clear_profile();
    for (hipEvent_t e : ctx->c.event_pool) (void)hipEventDestroy(e);
    ctx->c.event_pool.clear();
    ctx->c.plans.clear();
    if (ctx->c.host_scalars) (void)hipHostFree(ctx->c.host_scalars);
    delete ctx;
    return BSM_OK;
    BSM_API_END
}

int bsm_ctx_set_rows_per_wave(bsm_ctx ctx, int rows)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    BSM_REQUIRE(rows == 0 || rows == 2 || rows == 4 || rows == 8, BSM_EINVAL, "rows must be 0, 2, 4 or 8");
    BSM_HIP_TRY(hipStreamSynchronize(ctx->c.stream));
    // timing records point at plans: fold them away before the plans go
    ctx->c.retire_profile([](const Plan *) { return true; });
    ctx->c.plans.clear();
    ctx->c.rows_per_wave = rows;
    return BSM_OK;
    BSM_API_END
}

int bsm_ctx_set_product_variant(bsm_ctx ctx, int variant)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    BSM_REQUIRE(variant >= -1 && variant <= 6, BSM_EINVAL, "variant must be -1 .. 6");
    BSM_HIP_TRY(hipStreamSynchronize(ctx->c.stream));
    ctx->c.retire_profile([](const Plan *) { return true; });
    ctx->c.plans.clear();
    ctx->c.product_variant = variant;
    return BSM_OK;
    BSM_API_END
}

int bsm_ctx_set_group_span(bsm_ctx ctx, int span)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    BSM_REQUIRE(span >= 1 && span <= 4096, BSM_EINVAL, "span must be in 1..4096");
    BSM_HIP_TRY(hipStreamSynchronize(ctx->c.stream));
    ctx->c.retire_profile([](const Plan *) { return true; });
    ctx->c.plans.clear();
    ctx->c.group_span = span;
    return BSM_OK;
    BSM_API_END
}

int bsm_ctx_set_column_order(bsm_ctx ctx, int order)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    BSM_REQUIRE(order == 0 || order == 1, BSM_EINVAL, "column order must be 0 or 1");
    BSM_HIP_TRY(hipStreamSynchronize(ctx->c.stream));
    ctx->c.retire_profile([](const Plan *) { return true; });
    ctx->c.plans.clear();
    ctx->c.column_order = order;
    return BSM_OK;
    BSM_API_END
}

int bsm_ctx_set_transposed_plans(bsm_ctx ctx, int mode)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    BSM_REQUIRE(mode >= 0 && mode <= 2, BSM_EINVAL, "mode must be 0, 1 or 2");
    BSM_HIP_TRY(hipStreamSynchronize(ctx->c.stream));
    ctx->c.retire_profile([](const Plan *) { return true; });
    ctx->c.plans.clear();
    ctx->c.transposed_plans = mode;
    return BSM_OK;
    BSM_API_END
}

int bsm_ctx_set_profiling(bsm_ctx ctx, int enable)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    if (enable) {
        BSM_HIP_TRY(hipStreamSynchronize(ctx->c.stream));
        ctx->c.clear_profile();
        ctx->c.retired.clear();
    }
    ctx->c.profiling = enable != 0;
    return BSM_OK;
    BSM_API_END
}

int bsm_ctx_product_stats(bsm_ctx ctx, bsm_product_stat *out, int max, int *count)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr && count != nullptr && (out != nullptr || max == 0), BSM_EINVAL, "NULL argument");
    Context &c = ctx->c;
    BSM_HIP_TRY(hipStreamSynchronize(c.stream));
    auto agg = c.retired;
    for (auto &r : c.prof) {
        float ms = 0.f;
        BSM_HIP_TRY(hipEventElapsedTime(&ms, r.start, r.stop));
        auto &acc = agg[Context::prof_key(r)];
        acc.launches += 1;
        acc.flops += r.plan->flops * r.products;
        acc.ms += ms;
    }
    std::vector<bsm_product_stat> v;
    for (auto &kv : agg) {
        bsm_product_stat s{};
        s.natoms = std::get<0>(kv.first);
        s.b = std::get<1>(kv.first);
        s.cutoff_a = std::get<2>(kv.first);
        s.cutoff_b = std::get<3>(kv.first);
        s.cutoff_c = std::get<4>(kv.first);
        s.variant = std::get<5>(kv.first);
        s.rows = std::get<6>(kv.first);
        s.precision = std::get<7>(kv.first);
        s.products = std::get<8>(kv.first);
        s.launches = kv.second.launches;
        s.flops = kv.second.flops;
        s.ms = kv.second.ms;
        v.push_back(s);
    }
    std::sort(v.begin(), v.end(), [](const bsm_product_stat &a, const bsm_product_stat &b) { return a.ms > b.ms; });
    *count = (int)v.size();
    for (int n = 0; n < max && n < (int)v.size(); ++n) out[n] = v[n];
    return BSM_OK;
    BSM_API_END
}

int bsm_ctx_set_stream(bsm_ctx ctx, void *hip_stream)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    ctx->c.stream = (hipStream_t)hip_stream;
    return BSM_OK;
    BSM_API_END
}

int bsm_create_pattern(bsm_ctx ctx, int natoms, int b, const double *pos, const double box[3], double cutoff,
                       bsm_pattern *out)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr && out != nullptr && box != nullptr, BSM_EINVAL, "NULL argument");
    *out = make_pattern(&ctx->c, natoms, b, pos, box, cutoff);
    return BSM_OK;
    BSM_API_END
}

int bsm_pattern_destroy(bsm_pattern p)
{
    BSM_API_BEGIN
    destroy_pattern(p);
    return BSM_OK;
    BSM_API_END
}

int bsm_pattern_get_info(bsm_pattern p, bsm_pattern_info *out)
{
    BSM_API_BEGIN
    BSM_REQUIRE(p != nullptr && out != nullptr, BSM_EINVAL, "NULL argument");
    out->natoms = p->natoms;
    out->b = p->b;
    out->nnzb = p->nnzb;
    out->max_row = p->max_row;
    out->cutoff = p->cutoff;
    for (int d = 0; d < 3; ++d) out->box[d] = p->box[d];
    out->rowptr = p->rowptr.as<int32_t>();
    out->cols = p->cols.as<int32_t>();
    out->tmap = p->tmap.as<int32_t>();
    out->diag = p->diag.as<int32_t>();
    out->pos = p->pos.as<double>();
    return BSM_OK;
    BSM_API_END
}

int bsm_pattern_copy_to_host(bsm_pattern p, int32_t *rowptr_host, int32_t *cols_host)
{
    BSM_API_BEGIN
    BSM_REQUIRE(p != nullptr && rowptr_host != nullptr && cols_host != nullptr, BSM_EINVAL, "NULL argument");
    hipStream_t st = p->ctx->stream;
    BSM_HIP_TRY(hipMemcpyAsync(rowptr_host, p->rowptr.ptr, sizeof(int32_t) * (p->natoms + 1),
                               hipMemcpyDeviceToHost, st));
    if (p->nnzb > 0)
        BSM_HIP_TRY(hipMemcpyAsync(cols_host, p->cols.ptr, sizeof(int32_t) * p->nnzb, hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    return BSM_OK;
    BSM_API_END
}

int bsm_matrix_fill_blocks(bsm_ctx ctx, const bsm_matrix *M, int64_t count, const int32_t *rows,
                           const int32_t *cols, const double *blocks)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    check_matrix(M, "M");
    BSM_REQUIRE(count >= 0, BSM_EINVAL, "count is negative");
    BSM_REQUIRE(count == 0 || (rows && cols && blocks), BSM_EINVAL, "NULL block arrays");
    fill_blocks(&ctx->c, M->pattern, (double *)M->blocks, count, rows, cols, blocks);
    return BSM_OK;
    BSM_API_END
}

int bsm_axpby(bsm_ctx ctx, double alpha, const bsm_matrix *X, double beta, const bsm_matrix *Y)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    check_matrix(X, "X");
    check_matrix(Y, "Y");
    BSM_REQUIRE(X->pattern == Y->pattern, BSM_EPATTERN, "X and Y must share a pattern");
    axpby(&ctx->c, nelems(X->pattern), alpha, (const double *)X->blocks, beta, (double *)Y->blocks);
    return BSM_OK;
    BSM_API_END
}

int bsm_symmetrize(bsm_ctx ctx, const bsm_matrix *M)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    check_matrix(M, "M");
    symmetrize(&ctx->c, M->pattern, (double *)M->blocks);
    return BSM_OK;
    BSM_API_END
}

int bsm_mask_copy(bsm_ctx ctx, const bsm_matrix *src, const bsm_matrix *dst)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    check_matrix(src, "src");
    check_matrix(dst, "dst");
    check_same_shape(src, dst);
    BSM_REQUIRE(!overlaps(src, dst), BSM_EINVAL, "src and dst overlap");
    mask_copy(&ctx->c, src->pattern, (const double *)src->blocks, dst->pattern, (double *)dst->blocks);
    return BSM_OK;
    BSM_API_END
}

int bsm_set_identity(bsm_ctx ctx, const bsm_matrix *M, double alpha)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    check_matrix(M, "M");
    set_identity(&ctx->c, M->pattern, alpha, (double *)M->blocks);
    return BSM_OK;
    BSM_API_END
}

int bsm_dot(bsm_ctx ctx, const bsm_matrix *A, const bsm_matrix *B, double *out)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr && out != nullptr, BSM_EINVAL, "NULL argument");
    check_matrix(A, "A");
    check_matrix(B, "B");
    BSM_REQUIRE(A->pattern == B->pattern, BSM_EPATTERN, "A and B must share a pattern");
    const double *a = (const double *)A->blocks, *b = (const double *)B->blocks;
    dots(&ctx->c, 1, A->pattern, &a, &b, out);
    if (!std::isfinite(*out)) return fail(BSM_ENONFINITE, "inner product is not finite");
    return BSM_OK;
    BSM_API_END
}

int bsm_multiply_truncate(bsm_ctx ctx, double alpha, const bsm_matrix *A, const bsm_matrix *B, double beta,
                          const bsm_matrix *C)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    check_matrix(A, "A");
    check_matrix(B, "B");
    check_matrix(C, "C");
    check_same_shape(A, B);
    check_same_shape(A, C);
    BSM_REQUIRE(!overlaps(C, A) && !overlaps(C, B), BSM_EINVAL, "C overlaps A or B");
    Plan *plan = get_plan(&ctx->c, A->pattern, B->pattern, C->pattern);
    launch_product_f64(&ctx->c, plan, alpha, A->pattern, (const double *)A->blocks, B->pattern,
                       (const double *)B->blocks, beta, C->pattern, (double *)C->blocks);
    return BSM_OK;
    BSM_API_END
}

int bsm_multiply_truncate_pair(bsm_ctx ctx, double alpha, const bsm_matrix *A, const bsm_matrix *A2,
                               const bsm_matrix *B, double beta, const bsm_matrix *C, const bsm_matrix *C2)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    check_matrix(A, "A");
    check_matrix(A2, "A2");
    check_matrix(B, "B");
    check_matrix(C, "C");
    check_matrix(C2, "C2");
    check_same_shape(A, B);
    check_same_shape(A, C);
    BSM_REQUIRE(A2->pattern == A->pattern, BSM_EPATTERN, "A2 must lie on A's pattern");
    BSM_REQUIRE(C2->pattern == C->pattern, BSM_EPATTERN, "C2 must lie on C's pattern");
    BSM_REQUIRE(!overlaps(C, A) && !overlaps(C, A2) && !overlaps(C, B) && !overlaps(C2, A) &&
                    !overlaps(C2, A2) && !overlaps(C2, B) && !overlaps(C, C2),
                BSM_EINVAL, "C or C2 overlaps an operand or each other");
    Context *c = &ctx->c;
    Plan *pair = get_pair_plan(c, A->pattern, B->pattern, C->pattern);
    if (pair) {
        launch_product_pair_f64(c, pair, alpha, A->pattern, (const double *)A->blocks, (const double *)A2->blocks,
                                B->pattern, (const double *)B->blocks, beta, C->pattern, (double *)C->blocks,
                                (double *)C2->blocks);
    } else {
        Plan *plan = get_plan(c, A->pattern, B->pattern, C->pattern);
        launch_product_f64(c, plan, alpha, A->pattern, (const double *)A->blocks, B->pattern,
                           (const double *)B->blocks, beta, C->pattern, (double *)C->blocks);
        launch_product_f64(c, plan, alpha, A->pattern, (const double *)A2->blocks, B->pattern,
                           (const double *)B->blocks, beta, C->pattern, (double *)C2->blocks);
    }
    return BSM_OK;
    BSM_API_END
}

int bsm_multiply_truncate_pair_a(bsm_ctx ctx, double alpha, const bsm_matrix *A, const bsm_matrix *B,
                                 const bsm_matrix *B2, double beta, const bsm_matrix *C, const bsm_matrix *C2)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    check_matrix(A, "A");
    check_matrix(B, "B");
    check_matrix(B2, "B2");
    check_matrix(C, "C");
    check_matrix(C2, "C2");
    check_same_shape(A, B);
    check_same_shape(A, C);
    BSM_REQUIRE(B2->pattern == B->pattern, BSM_EPATTERN, "B2 must lie on B's pattern");
    BSM_REQUIRE(C2->pattern == C->pattern, BSM_EPATTERN, "C2 must lie on C's pattern");
    BSM_REQUIRE(!overlaps(C, A) && !overlaps(C, B) && !overlaps(C, B2) && !overlaps(C2, A) &&
                    !overlaps(C2, B) && !overlaps(C2, B2) && !overlaps(C, C2),
                BSM_EINVAL, "C or C2 overlaps an operand or each other");
    Context *c = &ctx->c;
    Plan *pair = get_pair_plan_a(c, A->pattern, B->pattern, C->pattern);
    if (pair) {
        launch_product_pair_a_f64(c, pair, alpha, A->pattern, (const double *)A->blocks, B->pattern,
                                  (const double *)B->blocks, (const double *)B2->blocks, beta, C->pattern,
                                  (double *)C->blocks, (double *)C2->blocks);
    } else {
        Plan *plan = get_plan(c, A->pattern, B->pattern, C->pattern);
        launch_product_f64(c, plan, alpha, A->pattern, (const double *)A->blocks, B->pattern,
                           (const double *)B->blocks, beta, C->pattern, (double *)C->blocks);
        launch_product_f64(c, plan, alpha, A->pattern, (const double *)A->blocks, B->pattern,
                           (const double *)B2->blocks, beta, C->pattern, (double *)C2->blocks);
    }
    return BSM_OK;
    BSM_API_END
}

int bsm_multiply_truncate_prec(bsm_ctx ctx, int precision, double alpha, const bsm_matrix *A,
                               const bsm_matrix *B, double beta, const bsm_matrix *C)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr, BSM_EINVAL, "ctx is NULL");
    check_matrix(A, "A");
    check_matrix(B, "B");
    check_matrix(C, "C");
    check_same_shape(A, B);
    check_same_shape(A, C);
    BSM_REQUIRE(!overlaps(C, A) && !overlaps(C, B), BSM_EINVAL, "C overlaps A or B");
    Plan *plan = get_plan(&ctx->c, A->pattern, B->pattern, C->pattern);
    launch_product_mixed(&ctx->c, plan, precision, alpha, A->pattern, (const double *)A->blocks, B->pattern,
                         (const double *)B->blocks, beta, C->pattern, (double *)C->blocks);
    return BSM_OK;
    BSM_API_END
}

int bsm_product_flops(bsm_ctx ctx, bsm_pattern PA, bsm_pattern PB, bsm_pattern PC, double *flops)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx && PA && PB && PC && flops, BSM_EINVAL, "NULL argument");
    BSM_REQUIRE(PA->natoms == PB->natoms && PA->natoms == PC->natoms && PA->b == PB->b && PA->b == PC->b,
                BSM_EPATTERN, "atom count or orbitals per atom differ");
    *flops = get_plan(&ctx->c, PA, PB, PC)->flops;
    return BSM_OK;
    BSM_API_END
}

int bsm_trace_product(bsm_ctx ctx, const bsm_matrix *A, const bsm_matrix *B, double *out)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr && out != nullptr, BSM_EINVAL, "NULL argument");
    check_matrix(A, "A");
    check_matrix(B, "B");
    check_same_shape(A, B);
    const double *a = (const double *)A->blocks, *b = (const double *)B->blocks;
    trace_products(&ctx->c, 1, A->pattern, &a, B->pattern, &b, out);
    if (!std::isfinite(*out)) return fail(BSM_ENONFINITE, "trace is not finite");
    return BSM_OK;
    BSM_API_END
}

int bsm_trace_product_noalloc(bsm_ctx ctx, const bsm_matrix *A, const bsm_matrix *B, double *out_dev)
{
    BSM_API_BEGIN
    BSM_REQUIRE(ctx != nullptr && out_dev != nullptr, BSM_EINVAL, "NULL argument");
    check_matrix(A, "A");
    check_matrix(B, "B");
    check_same_shape(A, B);
    trace_product_noalloc(&ctx->c, A->pattern, (const double *)A->blocks, B->pattern, (const double *)B->blocks,
                          out_dev);
    return BSM_OK;
    BSM_API_END
}

}  // extern "C"
