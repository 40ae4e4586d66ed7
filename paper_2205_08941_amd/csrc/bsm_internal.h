// Internal declarations shared by the host drivers and the HIP kernels of libbsm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bsm.h"

namespace bsm {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define BSM_HIP_TRY(expr)                                                              \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess)                                                          \
            throw ::bsm::Error{BSM_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
    } while (0)

#define BSM_REQUIRE(cond, code, msg)                                                   \
    do {                                                                               \
        if (!(cond)) throw ::bsm::Error{(code), (msg)};                                \
    } while (0)

// ---------------------------------------------------------------- memory
class Context;

// Device buffer from the context allocator; frees on destruction.
struct DevBuf {
    Context *ctx = nullptr;
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(Context *c, size_t n);
    ~DevBuf();
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept;
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Product plan for C = mask_{P_C}(A B): tiles of (G rows, up to jt output
// columns) and, per tile, the list of k with the slots of A_{i_a k} and B_kj.
// Built on the GPU on first use, cached per (P_A, P_B, P_C).
struct Plan {
    uint64_t ids[3] = {0, 0, 0};
    double cutoffs[3] = {0, 0, 0};
    int natoms = 0, b = 0;
    int G = 0;                  // rows per wavefront tile
    int variant = 0;            // 0: A through SGPRs, 1: A in VGPRs with DPP broadcast, 2: workgroup tiles,
                                // 3, 4: LDS-DMA rings, 5: rings with tiles shared by two waves
    int waves = 1;              // waves per tile (2 for variant 5)
    int transposed = 0;         // 1: computes C^T = B^T A^T (operands swapped, blocks read and C written transposed)
    int jt = 0;                 // output block columns per tile (waves * 64 / b)
    int64_t ntiles = 0;
    int64_t nentries = 0;
    int span = 1;               // row groups interleaved in the launch order
    DevBuf order;               // int [ntiles]: launch slot -> tile
    DevBuf hdr;                 // int [ntiles][G + G*jt]: rows, C slots
    DevBuf ebeg;                // int64 [ntiles + 1]: entry ranges
    DevBuf ent;                 // int [nentries][waves * G + jt]: per wave A slots, then its B slots
    double flops = 0.0;         // algorithmic: 2 b^3 per block triple
    int64_t triples = 0;
    int64_t rowwork = 0;        // rows multiplied, summed over entries (and waves)
};

class Context {
  public:
    int device = 0;
    hipStream_t stream = nullptr;
    bsm_alloc_fn alloc_fn = nullptr;
    bsm_free_fn free_fn = nullptr;
    void *user = nullptr;
    uint64_t next_pattern_id = 1;
    int rows_per_wave = 0;      // product plans: 0 = per-b default, else 2, 4 or 8
    int product_variant = -1;   // product kernel variant of plans built from now on (-1: per-b default)
    int group_span = 4;         // row groups interleaved in product launch order
    int column_order = 1;       // tile columns: 0 ascending, 1 grouped by the rows they hold outputs for
    // derived patterns (same atoms, another cutoff), owned here, keyed by (source id, cutoff)
    std::map<std::pair<uint64_t, double>, bsm_pattern_s *> derived;
    // (A, B, C, variant, rows, transposed plans allowed)
    std::map<std::tuple<uint64_t, uint64_t, uint64_t, int, int, int>, std::unique_ptr<Plan>> plans;
    int transposed_plans = 1;   // 0 never, 1 when estimated cheaper, 2 whenever allowed
    // reduction scratch
    DevBuf red_partials;        // double[kRedBlocks * kRedSlots]
    DevBuf err_flag;            // int
    DevBuf zero_block;          // 16 x 16 FP64 zeros (absent B blocks in the DPP product)
    double *host_scalars = nullptr;  // pinned host, kRedSlots doubles
    // product timing (bsm_ctx_set_profiling)
    struct ProfRec {
        const Plan *plan;
        hipEvent_t start, stop;
        int prec;               // BSM_F64, BSM_F32 or BSM_BF16
        int products = 1;       // 2: a paired launch (two products on one plan)
    };
    // statistics class: (natoms, b, cutoffs A, B, C, kernel variant, rows per tile, precision,
    // products per launch)
    using ProfKey = std::tuple<int, int, double, double, double, int, int, int, int>;
    static ProfKey prof_key(const ProfRec &r)
    {
        return ProfKey(r.plan->natoms, r.plan->b, r.plan->cutoffs[0], r.plan->cutoffs[1], r.plan->cutoffs[2],
                       r.plan->variant, r.plan->G, r.prec, r.products);
    }
    bool profiling = false;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> event_pool;
    struct ProfAcc {
        int64_t launches = 0;
        double flops = 0.0, ms = 0.0;
    };
    // launches of plans whose patterns were destroyed while profiling
    std::map<ProfKey, ProfAcc> retired;
    // FP32 operand copies for mixed-precision products (grown on demand)
    DevBuf f32buf[2];
    float *scratch_f32(int which, int64_t n);
    hipEvent_t take_event();
    void clear_profile();
    // fold timing records of the picked plans into `retired` (they are about to go)
    void retire_profile(const std::function<bool(const Plan *)> &pick);

    void *allocate(size_t bytes);
    void release(void *p);
    void forget_pattern(uint64_t id);
};

static constexpr int kRedBlocks = 1024;   // fixed grid for deterministic reductions
static constexpr int kRedSlots = 16;      // traces computed by one fused launch, at most

}  // namespace bsm

struct bsm_ctx_s {
    bsm::Context c;
};

struct bsm_pattern_s {
    bsm::Context *ctx = nullptr;
    uint64_t id = 0;
    int natoms = 0, b = 0, max_row = 0;
    int64_t nnzb = 0;
    double cutoff = 0.0;
    double box[3] = {0, 0, 0};
    bsm::DevBuf pos, rowptr, cols, tmap, diag, rowidx;   // rowidx: row of every slot
};

namespace bsm {

// ---------------------------------------------------------------- helpers
int64_t nelems(const bsm_pattern_s *p);
void check_matrix(const bsm_matrix *M, const char *name);
void check_same_shape(const bsm_matrix *A, const bsm_matrix *B);
bsm_pattern_s *make_pattern(Context *ctx, int natoms, int b, const double *pos_dev,
                            const double box[3], double cutoff);
// A pattern over the same atoms with another cutoff (owned by the caller).
bsm_pattern_s *derived_pattern(const bsm_pattern_s *p, double cutoff);
// The same, cached in (and owned by) the context until the source pattern or the
// context is destroyed, so repeated driver calls reuse patterns and plans.
const bsm_pattern_s *derived_pattern_cached(const bsm_pattern_s *p, double cutoff);
void destroy_pattern(bsm_pattern_s *p);
Plan *get_plan(Context *ctx, const bsm_pattern_s *A, const bsm_pattern_s *B, const bsm_pattern_s *C);
// A plan of a given kernel variant (0: SGPR, 1: DPP wave tiles, 2: workgroup tiles, 3 and 4: LDS-DMA
// rings, 5: rings with tiles shared by two waves, 6: ring tiles on the FP64 matrix cores) and rows
// per tile; transposed plans only where allowed (variant 4 launches).
Plan *get_plan_kind(Context *ctx, const bsm_pattern_s *A, const bsm_pattern_s *B, const bsm_pattern_s *C,
                    int variant, int G, bool allow_transposed = false);

// ---------------------------------------------------------------- launches
void launch_product_f64(Context *ctx, const Plan *plan, double alpha, const bsm_pattern_s *PA,
                        const double *A, const bsm_pattern_s *PB, const double *B, double beta,
                        const bsm_pattern_s *PC, double *C);
// The plan of a paired FP64 launch (C = alpha A B + beta C and C2 = alpha A2 B + beta C2, A and A2
// on PA): direct one-wave ring tiles of 4 rows, the pair run as 8-row tiles; nullptr when the
// pair cannot run as one launch (b other than 4 and 9, or another kernel variant chosen).
Plan *get_pair_plan(Context *ctx, const bsm_pattern_s *PA, const bsm_pattern_s *PB, const bsm_pattern_s *PC);
void launch_product_pair_f64(Context *ctx, const Plan *plan, double alpha, const bsm_pattern_s *PA,
                             const double *A, const double *A2, const bsm_pattern_s *PB, const double *B,
                             double beta, const bsm_pattern_s *PC, double *C, double *C2);
// The same for two products sharing their left operand (C = alpha A B + beta C and C2 = alpha A B2 +
// beta C2, B and B2 on PB), on a transposed 4-row plan (C = (B^T A^T)^T); nullptr as above.
Plan *get_pair_plan_a(Context *ctx, const bsm_pattern_s *PA, const bsm_pattern_s *PB, const bsm_pattern_s *PC);
void launch_product_pair_a_f64(Context *ctx, const Plan *plan, double alpha, const bsm_pattern_s *PA,
                               const double *A, const bsm_pattern_s *PB, const double *B, const double *B2,
                               double beta, const bsm_pattern_s *PC, double *C, double *C2);
// A transposed ring plan (variant 4) of G rows, cached apart from the plans get_plan_kind picks.
Plan *get_transposed_plan(Context *ctx, const bsm_pattern_s *A, const bsm_pattern_s *B, const bsm_pattern_s *C, int G);
void build_plan(Context *ctx, const bsm_pattern_s *PA, const bsm_pattern_s *PB, const bsm_pattern_s *PC,
                Plan *plan, int G, int waves, int transposed = 0);
// prec BSM_F64: the FP64 product; BSM_F32 / BSM_BF16: operands rounded to that
// precision, FP32 accumulation, FP64 result.
void launch_product_mixed(Context *ctx, const Plan *plan, int prec, double alpha, const bsm_pattern_s *PA,
                          const double *A, const bsm_pattern_s *PB, const double *B, double beta,
                          const bsm_pattern_s *PC, double *C);
int default_rows_per_wave(int b);

// Traces of products Tr(A_n B_n) for up to kRedSlots pairs in one pass; A_n all
// on one pattern, B_n all on one pattern.  Results to host `out`.  Synchronises.
void trace_products(Context *ctx, int count, const bsm_pattern_s *PA, const double *const *A,
                    const bsm_pattern_s *PB, const double *const *B, double *out);
// The LNV's fixed trace sets on one pattern, from the distinct matrices only
// (each loaded once): kTracesEnergy, A = {X, W}, B = {Y, X}: Tr XY, Tr WY,
// Tr XX, Tr WX; kTracesLineSearch, A = {X_D, X, M1, W, Q}, B = {Y, Y_D, X_D, X}:
// the 15 traces of the line-search polynomials.  Same bits as trace_products.
enum { kTracesEnergy = 0, kTracesLineSearch = 1 };
void trace_set(Context *ctx, int kind, const bsm_pattern_s *P, const double *const *A, const double *const *B,
               double *out);
// <A_n, B_n> (same pattern) for up to kRedSlots pairs.  Synchronises.
void dots(Context *ctx, int count, const bsm_pattern_s *P, const double *const *A,
          const double *const *B, double *out);
double trace_single(Context *ctx, const bsm_pattern_s *P, const double *A);
// Address of the allocation-free trace's static scratch on `device` (the current
// device), taken once per device; called by bsm_ctx_create.
void trace_scratch_setup(int device);
// Tr(A B) into *out_dev (device memory), asynchronous, partial sums in the static
// scratch: no allocation and no synchronisation.
void trace_product_noalloc(Context *ctx, const bsm_pattern_s *PA, const double *A, const bsm_pattern_s *PB,
                           const double *B, double *out_dev);
double max_abs_row_sum(Context *ctx, const bsm_pattern_s *P, const double *A);
// ||A - I||_F^2, elementwise.  Synchronises.
double dist_identity_sq(Context *ctx, const bsm_pattern_s *P, const double *A);

void axpby(Context *ctx, int64_t n, double alpha, const double *x, double beta, double *y);
// z <- a x + b y + c z (z may be x or y elementwise-aliased: per-element update)
void axpbypcz(Context *ctx, int64_t n, double a, const double *x, double b, const double *y,
              double c, double *z);
void symmetrize(Context *ctx, const bsm_pattern_s *P, double *M);
// out <- alpha (M + M^T) + beta out; out must not alias M
void add_transpose(Context *ctx, const bsm_pattern_s *P, double alpha, const double *M, double beta,
                   double *out);
void mask_copy(Context *ctx, const bsm_pattern_s *Psrc, const double *src, const bsm_pattern_s *Pdst,
               double *dst);
void set_identity(Context *ctx, const bsm_pattern_s *P, double alpha, double *M);
void fill_blocks(Context *ctx, const bsm_pattern_s *P, double *M, int64_t count, const int32_t *rows,
                 const int32_t *cols, const double *blocks);

}  // namespace bsm
