// Spatial-cutoff patterns: GPU cell-list neighbour search -> block CSR with
// sorted columns, transpose map and diagonal slots.
//
// The pattern is the locality structure of the paper's sparse matrices
// (Background and Current Status): an atom block (i, j) exists only when the
// minimum-image distance of atoms i and j is below the range of the operator.
#include "bsm_internal.h"

#include <algorithm>
#include <climits>
#include <cmath>

namespace bsm {
namespace {

constexpr int kMaxRow = 8192;   // longest row the LDS row sort handles

// Squared minimum-image distance, rounded exactly as written (no FMA), so the
// strict d^2 < r^2 decision is the one a plain CPU evaluation makes.
__device__ inline double min_image_d2(const double *__restrict__ pos, double bx, double by,
                                      double bz, int i, int j)
{
#pragma clang fp contract(off)
    const double box[3] = {bx, by, bz};
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double d = pos[3 * j + c] - pos[3 * i + c];
        double s = __builtin_rint(d / box[c]);
        d = d - s * box[c];
        d2 = d2 + d * d;
    }
    return d2;
}

struct Grid {
    int nc[3];
    int noff[3];   // neighbour offsets scanned per axis: 1, 2 or 3
    double box[3];
};

__device__ inline int cell_coord(double x, double box, int nc)
{
    double f = x / box;
    f -= floor(f);
    int c = (int)(f * nc);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_cell_index(int n, const double *__restrict__ pos, Grid g, int *__restrict__ cell,
                             int *__restrict__ cellcount, int *__restrict__ nonfinite)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!isfinite(pos[3 * i]) || !isfinite(pos[3 * i + 1]) || !isfinite(pos[3 * i + 2]))
        atomicOr(nonfinite, 1);
    int cx = cell_coord(pos[3 * i + 0], g.box[0], g.nc[0]);
    int cy = cell_coord(pos[3 * i + 1], g.box[1], g.nc[1]);
    int cz = cell_coord(pos[3 * i + 2], g.box[2], g.nc[2]);
    int c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
    cell[i] = c;
    atomicAdd(&cellcount[c], 1);
}

// Exclusive scan of n ints into out[0..n] (out[n] = total) by one workgroup.
// Sets *overflow when the total does not fit in int32.
__global__ __launch_bounds__(1024) void k_scan(int n, const int *__restrict__ in, int *__restrict__ out,
                                               int *__restrict__ overflow)
{
    __shared__ long long part[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    const int chunk = (n + nt - 1) / nt;
    const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
    long long s = 0;
    for (int k = lo; k < hi; ++k) s += in[k];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {   // Hillis-Steele inclusive scan
        long long v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long run = part[t] - s;
    for (int k = lo; k < hi; ++k) {
        out[k] = (int)run;
        run += in[k];
    }
    if (t == nt - 1) {
        out[n] = (int)part[t];
        *overflow = part[t] > (long long)INT_MAX ? 1 : 0;
    }
}

__global__ void k_cell_scatter(int n, const int *__restrict__ cell, const int *__restrict__ cellstart,
                               int *__restrict__ cellfill, int *__restrict__ cellatoms)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell[i];
    cellatoms[cellstart[c] + atomicAdd(&cellfill[c], 1)] = i;
}

// One thread per atom: visit the neighbour cells, count (mode 0) or write
// (mode 1) the columns j with d^2 < r^2 (and j == i).
template <int MODE>
__global__ void k_neighbors(int n, const double *__restrict__ pos, Grid g, double r2,
                            const int *__restrict__ cell, const int *__restrict__ cellstart,
                            const int *__restrict__ cellatoms, int *__restrict__ rowcount,
                            const int *__restrict__ rowptr, int *__restrict__ cols)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell[i];
    int cz = c % g.nc[2], cy = (c / g.nc[2]) % g.nc[1], cx = c / (g.nc[2] * g.nc[1]);
    int cnt = 0;
    int w = (MODE == 1) ? rowptr[i] : 0;
    for (int ox = 0; ox < g.noff[0]; ++ox) {
        int ax = (g.noff[0] == 3) ? cx + ox - 1 : cx + ox;
        ax = ((ax % g.nc[0]) + g.nc[0]) % g.nc[0];
        for (int oy = 0; oy < g.noff[1]; ++oy) {
            int ay = (g.noff[1] == 3) ? cy + oy - 1 : cy + oy;
            ay = ((ay % g.nc[1]) + g.nc[1]) % g.nc[1];
            for (int oz = 0; oz < g.noff[2]; ++oz) {
                int az = (g.noff[2] == 3) ? cz + oz - 1 : cz + oz;
                az = ((az % g.nc[2]) + g.nc[2]) % g.nc[2];
                int cc = (ax * g.nc[1] + ay) * g.nc[2] + az;
                for (int q = cellstart[cc]; q < cellstart[cc + 1]; ++q) {
                    int j = cellatoms[q];
                    if (j == i || min_image_d2(pos, g.box[0], g.box[1], g.box[2], i, j) < r2) {
                        if (MODE == 1) cols[w] = j;
                        ++w;
                        ++cnt;
                    }
                }
            }
        }
    }
    if (MODE == 0) rowcount[i] = cnt;
}

// One workgroup per row: bitonic sort of the row's columns in LDS.
__global__ __launch_bounds__(256) void k_sort_rows(int n, const int *__restrict__ rowptr,
                                                   int *__restrict__ cols)
{
    __shared__ int v[kMaxRow];
    int i = blockIdx.x;
    if (i >= n) return;
    int lo = rowptr[i], len = rowptr[i + 1] - lo;
    int p2 = 1;
    while (p2 < len) p2 <<= 1;
    for (int t = threadIdx.x; t < p2; t += blockDim.x) v[t] = (t < len) ? cols[lo + t] : INT_MAX;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int t = threadIdx.x; t < p2; t += blockDim.x) {
                int o = t ^ jj;
                if (o > t) {
                    bool up = (t & k) == 0;
                    int a = v[t], b = v[o];
                    if ((a > b) == up) {
                        v[t] = b;
                        v[o] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < len; t += blockDim.x) cols[lo + t] = v[t];
}

__device__ inline int find_in_row(const int *__restrict__ rowptr, const int *__restrict__ cols, int i,
                                  int j)
{
    int lo = rowptr[i], hi = rowptr[i + 1], end = hi;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cols[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && cols[lo] == j) ? lo : -1;
}

__global__ void k_rows_of_slots(int n, const int *__restrict__ rowptr, int *__restrict__ rowidx)
{
    int i = blockIdx.x;
    if (i >= n) return;
    for (int s = rowptr[i] + threadIdx.x; s < rowptr[i + 1]; s += blockDim.x) rowidx[s] = i;
}

__global__ void k_tmap(int64_t nnz, const int *__restrict__ rowptr, const int *__restrict__ cols,
                       const int *__restrict__ rowidx, int *__restrict__ tmap, int *__restrict__ bad)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nnz) return;
    int t = find_in_row(rowptr, cols, cols[s], rowidx[s]);
    tmap[s] = t;
    if (t < 0) atomicOr(bad, 1);
}

__global__ void k_diag(int n, const int *__restrict__ rowptr, const int *__restrict__ cols,
                       int *__restrict__ diag)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) diag[i] = find_in_row(rowptr, cols, i, i);
}

__global__ void k_max_row(int n, const int *__restrict__ rowptr, int *__restrict__ mx)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(mx, rowptr[i + 1] - rowptr[i]);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

bsm_pattern_s *make_pattern(Context *ctx, int natoms, int b, const double *pos_dev, const double box[3],
                            double cutoff)
{
    BSM_REQUIRE(natoms > 0, BSM_EINVAL, "natoms must be positive");
    BSM_REQUIRE(b >= 1 && b <= 16, BSM_EINVAL, "b must be in 1..16");
    BSM_REQUIRE(cutoff > 0 && std::isfinite(cutoff), BSM_EINVAL, "cutoff must be positive");
    BSM_REQUIRE(pos_dev != nullptr, BSM_EINVAL, "positions are NULL");
    for (int d = 0; d < 3; ++d)
        BSM_REQUIRE(box[d] > 0 && std::isfinite(box[d]), BSM_EINVAL, "box must be positive");

    hipStream_t st = ctx->stream;
    std::unique_ptr<bsm_pattern_s> p(new bsm_pattern_s());
    p->ctx = ctx;
    p->id = ctx->next_pattern_id++;
    p->natoms = natoms;
    p->b = b;
    p->cutoff = cutoff;
    for (int d = 0; d < 3; ++d) p->box[d] = box[d];
    p->pos = DevBuf(ctx, sizeof(double) * 3 * (size_t)natoms);
    BSM_HIP_TRY(hipMemcpyAsync(p->pos.ptr, pos_dev, sizeof(double) * 3 * (size_t)natoms,
                               hipMemcpyDeviceToDevice, st));

    Grid g;
    int64_t ncells = 1;
    for (int d = 0; d < 3; ++d) {
        double q = std::floor(box[d] / cutoff);
        int nc = (int)std::max(1.0, std::min(q, 256.0));
        g.nc[d] = nc;
        g.noff[d] = nc >= 3 ? 3 : nc;
        g.box[d] = box[d];
        ncells *= nc;
    }

    DevBuf cell(ctx, sizeof(int) * natoms), cellcount(ctx, sizeof(int) * ncells),
        cellstart(ctx, sizeof(int) * (ncells + 1)), cellfill(ctx, sizeof(int) * ncells),
        cellatoms(ctx, sizeof(int) * natoms), rowcount(ctx, sizeof(int) * natoms),
        flags(ctx, sizeof(int) * 8);
    BSM_HIP_TRY(hipMemsetAsync(cellcount.ptr, 0, sizeof(int) * ncells, st));
    BSM_HIP_TRY(hipMemsetAsync(cellfill.ptr, 0, sizeof(int) * ncells, st));
    BSM_HIP_TRY(hipMemsetAsync(flags.ptr, 0, sizeof(int) * 8, st));
    int *fl = flags.as<int>();

    k_cell_index<<<blocks_for(natoms, 256), 256, 0, st>>>(natoms, p->pos.as<double>(), g, cell.as<int>(),
                                                            cellcount.as<int>(), fl + 4);
    k_scan<<<1, 1024, 0, st>>>((int)ncells, cellcount.as<int>(), cellstart.as<int>(), fl + 0);
    k_cell_scatter<<<blocks_for(natoms, 256), 256, 0, st>>>(natoms, cell.as<int>(), cellstart.as<int>(),
                                                              cellfill.as<int>(), cellatoms.as<int>());
    double r2 = cutoff * cutoff;
    k_neighbors<0><<<blocks_for(natoms, 128), 128, 0, st>>>(natoms, p->pos.as<double>(), g, r2,
                                                            cell.as<int>(), cellstart.as<int>(),
                                                            cellatoms.as<int>(), rowcount.as<int>(),
                                                            nullptr, nullptr);
    p->rowptr = DevBuf(ctx, sizeof(int) * (natoms + 1));
    k_scan<<<1, 1024, 0, st>>>(natoms, rowcount.as<int>(), p->rowptr.as<int>(), fl + 1);
    k_max_row<<<blocks_for(natoms, 256), 256, 0, st>>>(natoms, p->rowptr.as<int>(), fl + 2);
    int hostv[5] = {0, 0, 0, 0, 0};
    int total = 0;
    BSM_HIP_TRY(hipMemcpyAsync(hostv, fl, sizeof(int) * 5, hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipMemcpyAsync(&total, p->rowptr.as<int>() + natoms, sizeof(int), hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    BSM_REQUIRE(hostv[4] == 0, BSM_EINVAL, "positions are not finite");
    BSM_REQUIRE(hostv[1] == 0, BSM_EINVAL, "pattern has more than 2^31-1 blocks");
    BSM_REQUIRE(hostv[2] <= kMaxRow, BSM_EINVAL, "a pattern row is longer than 8192 blocks");
    p->nnzb = total;
    p->max_row = hostv[2];

    p->cols = DevBuf(ctx, sizeof(int) * (size_t)total);
    k_neighbors<1><<<blocks_for(natoms, 128), 128, 0, st>>>(natoms, p->pos.as<double>(), g, r2,
                                                            cell.as<int>(), cellstart.as<int>(),
                                                            cellatoms.as<int>(), nullptr,
                                                            p->rowptr.as<int>(), p->cols.as<int>());
    k_sort_rows<<<natoms, 256, 0, st>>>(natoms, p->rowptr.as<int>(), p->cols.as<int>());

    p->rowidx = DevBuf(ctx, sizeof(int) * (size_t)total);
    k_rows_of_slots<<<natoms, 64, 0, st>>>(natoms, p->rowptr.as<int>(), p->rowidx.as<int>());
    p->tmap = DevBuf(ctx, sizeof(int) * (size_t)total);
    p->diag = DevBuf(ctx, sizeof(int) * natoms);
    k_tmap<<<blocks_for(total, 256), 256, 0, st>>>(total, p->rowptr.as<int>(), p->cols.as<int>(),
                                                   p->rowidx.as<int>(), p->tmap.as<int>(), fl + 3);
    k_diag<<<blocks_for(natoms, 256), 256, 0, st>>>(natoms, p->rowptr.as<int>(), p->cols.as<int>(),
                                                    p->diag.as<int>());
    int bad = 0;
    BSM_HIP_TRY(hipMemcpyAsync(&bad, fl + 3, sizeof(int), hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    BSM_REQUIRE(bad == 0, BSM_EINVAL, "pattern is not symmetric (non-finite positions?)");
    return p.release();
}

bsm_pattern_s *derived_pattern(const bsm_pattern_s *p, double cutoff)
{
    return make_pattern(p->ctx, p->natoms, p->b, p->pos.as<double>(), p->box, cutoff);
}

const bsm_pattern_s *derived_pattern_cached(const bsm_pattern_s *p, double cutoff)
{
    Context *ctx = p->ctx;
    auto key = std::make_pair(p->id, cutoff);
    auto it = ctx->derived.find(key);
    if (it != ctx->derived.end()) return it->second;
    bsm_pattern_s *d = derived_pattern(p, cutoff);
    ctx->derived[key] = d;
    return d;
}

void destroy_pattern(bsm_pattern_s *p)
{
    if (!p) return;
    Context *ctx = p->ctx;
    // patterns derived from this one go first
    std::vector<bsm_pattern_s *> kids;
    for (auto it = ctx->derived.begin(); it != ctx->derived.end();) {
        if (it->first.first == p->id) {
            kids.push_back(it->second);
            it = ctx->derived.erase(it);
        } else {
            ++it;
        }
    }
    for (bsm_pattern_s *k : kids) destroy_pattern(k);
    ctx->forget_pattern(p->id);
    delete p;
}

}  // namespace bsm
