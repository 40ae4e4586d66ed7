// Truncated block-sparse products C <- alpha mask_{P_C}(A B) + beta C in FP64.
//
// The products of atom-block matrices cut back to a spatial-cutoff pattern are
// the operations the paper's linear-scaling solver is built from (Background
// and Current Status) and the part it already started to move to GPUs
// (Meeting the Exascale Challenges).
//
// Work decomposition (gfx950, wave64, FP64 vector FMA):
//   * atoms are taken G at a time as a row group; the union of the group's
//     rows of P_C is cut into runs of JT = 64 / b columns.  A tile is (row
//     group, run); one wavefront owns one tile;
//   * lane l holds column c = l % b of the output blocks (i_a, j), j = run[l / b],
//     for all G rows i_a of the group: G x b FP64 accumulators per lane;
//   * the plan lists, per tile, every k for which some (i_a, k, j) triple
//     exists, with the slots of A_{i_a k} and B_kj.  The wave walks that list:
//     it loads the b x b block A_{i_a k} at a wave-uniform address through the
//     scalar cache (an SGPR operand broadcast to all lanes), each lane loads its
//     column of B_kj once and uses it for all G rows.  Exec masks drop lanes
//     whose (k, j) or (i_a, j) is absent, so only existing triples are summed,
//     in ascending k (deterministic);
//   * the next list entry and its B columns are loaded while the current one
//     is multiplied; tiles are mapped so that each XCD owns a contiguous range
//     of row groups (neighbouring rows share A and B blocks in its L2).
// No zero fill enters the flop count: 2 b^3 per triple (i, k, j) present.
#include "bsm_internal.h"
#include "tiles.h"

#include <algorithm>
#include <climits>
#include <utility>
#include <vector>

namespace bsm {
namespace {

constexpr int kXcd = 8;       // MI355X: 8 XCDs, workgroups dealt round-robin
constexpr int kWaves = 4;     // wavefronts (tiles) per workgroup
constexpr int kMaxRows = 16;  // rows of a tile, at most
constexpr int kPlanChunks = 4;   // planner threads per tile (chunks of the k range)

__device__ inline int64_t logical_workgroup(int64_t nwg_padded)
{
    const int64_t w = blockIdx.x;
    const int64_t per = nwg_padded / kXcd;
    return (w % kXcd) * per + w / kXcd;
}

// Tile header, ints: rows[G] (atom ids, -1 = padding), cslot[G][JT] (slot of
// (i_a, j) in C or -1).  Entries of tile t: ebeg[t] .. ebeg[t+1], each G + JT
// ints: aslot[G] (slot of (i_a, k) in A or -1), bslot[JT] (slot of (k, j) in B or -1).
template <int B, int G, class T>
__global__ __launch_bounds__(256) void k_product_sgpr(
    int64_t ntiles, int64_t nwg_padded, const int *__restrict__ order, const int *__restrict__ hdr,
    const int64_t *__restrict__ ebeg, const int *__restrict__ ent, const T *__restrict__ vA,
    const T *__restrict__ vB, double *__restrict__ vC, double alpha, double beta)
{
    const int64_t slot = logical_workgroup(nwg_padded) * kWaves + (threadIdx.x >> 6);
    if (slot >= ntiles) return;
    tile_sgpr<B, G, T>(order[slot], hdr, ebeg, ent, vA, vB, vC, alpha, beta);
}

template <int B, int G>
__global__ __launch_bounds__(256) void k_product_f64_dpp(
    int64_t ntiles, int64_t nwg_padded, const int *__restrict__ order, const int *__restrict__ hdr,
    const int64_t *__restrict__ ebeg, const int *__restrict__ ent, const double *__restrict__ vA,
    const double *__restrict__ vB, const double *__restrict__ zblk, double *__restrict__ vC, double alpha,
    double beta)
{
    const int64_t slot = logical_workgroup(nwg_padded) * kWaves + (threadIdx.x >> 6);
    if (slot >= ntiles) return;
    tile_dpp<B, G>(order[slot], hdr, ebeg, ent, vA, vB, zblk, vC, alpha, beta);
}

// One workgroup tile (16 rows x JT columns) per workgroup.
template <int B>
__global__ __launch_bounds__(256) void k_product_wg(
    int64_t ntiles, int64_t nwg_padded, const int *__restrict__ order, const int *__restrict__ hdr,
    const int64_t *__restrict__ ebeg, const int *__restrict__ ent, const double *__restrict__ vA,
    const double *__restrict__ vB, double *__restrict__ vC, double alpha, double beta)
{
    __shared__ double lds[2 * WgTile<B>::kStage];
    const int64_t t = logical_workgroup(nwg_padded);
    if (t >= ntiles) return;   // uniform over the workgroup
    tile_wg<B>(order[t], hdr, ebeg, ent, vA, vB, vC, alpha, beta, lds);
}

// One wave tile per one-wave workgroup, operands through a per-wave LDS ring
// (BUF: copied through buffer resources of a_bytes and b_bytes).
template <int B, int G, int D, class T = double, bool BUF = false, int W = 1, int TR = 0>
__global__ __launch_bounds__(64 * W) void k_product_ring(
    int64_t ntiles, int64_t nwg_padded, const int *__restrict__ order, const int *__restrict__ hdr,
    const int64_t *__restrict__ ebeg, const int *__restrict__ ent, const T *__restrict__ vA,
    const T *__restrict__ vB, const T *__restrict__ zblk, double *__restrict__ vC, double alpha, double beta,
    unsigned a_bytes, unsigned b_bytes)
{
    constexpr int kRing = D * RingEntry<B, G, T>::kBytes;   // per wave
    __shared__ __attribute__((aligned(16))) char ring[W * kRing];
    const int64_t t = logical_workgroup(nwg_padded);
    if (t >= ntiles) return;   // uniform over the workgroup
    const int w = W > 1 ? (int)(threadIdx.x >> 6) : 0;
    tile_ring<B, G, D, T, BUF, W, TR>(order[t], hdr, ebeg, ent, vA, vB, zblk, vC, alpha, beta,
                                      (lds_char_t *)ring + w * kRing, a_bytes, b_bytes);
}

// Two products sharing B and the patterns (C = A B, C2 = A2 B) on one plan of G / 2
// rows: one wave tile of G rows per one-wave workgroup, B's copies serving both
// (TR = 1: a transposed plan, the launch passing the shared left operand as B).
template <int B, int G, bool BUF, int TR = 0>
__global__ __launch_bounds__(64) void k_product_ring_pair(
    int64_t ntiles, int64_t nwg_padded, const int *__restrict__ order, const int *__restrict__ hdr,
    const int64_t *__restrict__ ebeg, const int *__restrict__ ent, const double *__restrict__ vA,
    const double *__restrict__ vA2, const double *__restrict__ vB, const double *__restrict__ zblk,
    double *__restrict__ vC, double *__restrict__ vC2, double alpha, double beta, unsigned a_bytes,
    unsigned a2_bytes, unsigned b_bytes)
{
    __shared__ __attribute__((aligned(16))) char ring[2 * RingEntry<B, G, double>::kBytes];
    const int64_t t = logical_workgroup(nwg_padded);
    if (t >= ntiles) return;
    tile_ring<B, G, 2, double, BUF, 1, TR, 2>(order[t], hdr, ebeg, ent, vA, vB, zblk, vC, alpha, beta,
                                             (lds_char_t *)ring, a_bytes, b_bytes, vA2, vC2, a2_bytes);
}

// FP64 matrix-core tiles (b = 9, G-row wave tiles, variant 6), one per one-wave workgroup.
template <int G, bool BUF>
__global__ __launch_bounds__(64) void k_product_mfma_f64(
    int64_t ntiles, int64_t nwg_padded, const int *__restrict__ order, const int *__restrict__ hdr,
    const int64_t *__restrict__ ebeg, const int *__restrict__ ent, const double *__restrict__ vA,
    const double *__restrict__ vB, const double *__restrict__ zblk, double *__restrict__ vC, double alpha,
    double beta, unsigned a_bytes, unsigned b_bytes)
{
    __shared__ __attribute__((aligned(16))) char ring[2 * RingEntry<9, G, double>::kBytes];
    const int64_t t = logical_workgroup(nwg_padded);
    if (t >= ntiles) return;
    tile_mfma_f64<G, BUF>(order[t], hdr, ebeg, ent, vA, vB, zblk, vC, alpha, beta, (lds_char_t *)ring, a_bytes,
                          b_bytes);
}

// ---------------------------------------------------------------- operand rounding
// FP64 -> FP32 (round to nearest even); for BF16, the FP32 value rounded again
// to 8 significant bits (nearest even, Inf kept, NaN kept quiet), stored as FP32.
__device__ inline float round_bf16(float x)
{
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) {
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);
        u &= 0xffff0000u;
    }
    return __uint_as_float(u);
}

__global__ void k_round_copy(int64_t n, const double *__restrict__ x, float *__restrict__ y, int bf16)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float f = (float)x[e];
    y[e] = bf16 ? round_bf16(f) : f;
}

// 9 x 9 FP64 blocks -> packed BF16 blocks of the matrix-core tiles: row p holds
// elements (p, m), m = 0..8, then 7 zeros (transpose: row p holds (m, p)).
// Rounding as k_round_copy: to FP32, then to BF16, both to nearest even.
__global__ void k_pack_bf16_blocks(int64_t nblk, const double *__restrict__ x, unsigned short *__restrict__ y,
                                   int transpose)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nblk * kPackedBlock) return;
    const int64_t blk = e / kPackedBlock;
    const int w = (int)(e - blk * kPackedBlock), p = w >> 4, m = w & 15;
    unsigned short v = 0;
    if (m < 9) {
        const double xv = x[blk * 81 + (transpose ? m * 9 + p : p * 9 + m)];
        v = (unsigned short)(__float_as_uint(round_bf16((float)xv)) >> 16);
    }
    y[e] = v;
}

// BF16 matrix-core product tiles (b = 9, G-row wave tiles), one per one-wave workgroup
// (BUF: packed operands copied through buffer resources of a_bytes and b_bytes).
template <int G, bool BUF>
__global__ __launch_bounds__(64) void k_product_mfma_bf16(
    int64_t ntiles, int64_t nwg_padded, const int *__restrict__ order, const int *__restrict__ hdr,
    const int64_t *__restrict__ ebeg, const int *__restrict__ ent, const unsigned short *__restrict__ pA,
    const unsigned short *__restrict__ pBt, const unsigned short *__restrict__ pz, double *__restrict__ vC,
    double alpha, double beta, unsigned a_bytes, unsigned b_bytes)
{
    __shared__ __attribute__((aligned(16))) char ring[4 * (G + 7) * kPackedBytes];
    const int64_t t = logical_workgroup(nwg_padded);
    if (t >= ntiles) return;
    tile_mfma_bf16<G, BUF>(order[t], hdr, ebeg, ent, pA, pBt, pz, vC, alpha, beta, (lds_char_t *)ring, a_bytes,
                           b_bytes);
}

// ---------------------------------------------------------------- planner
// One thread per row group: size of the union of the group's rows of P_C.
__global__ void k_group_union(int n, int G, const int *__restrict__ rpC, const int *__restrict__ cC,
                              int jt, int *__restrict__ ntile)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int ng = (n + G - 1) / G;
    if (g >= ng) return;
    int p[kMaxRows], pe[kMaxRows];
    const int i0 = g * G, gr = min(G, n - i0);
    for (int a = 0; a < gr; ++a) {
        p[a] = rpC[i0 + a];
        pe[a] = rpC[i0 + a + 1];
    }
    int cnt = 0;
    while (true) {
        int m = 0x7fffffff;
        for (int a = 0; a < gr; ++a)
            if (p[a] < pe[a]) m = min(m, cC[p[a]]);
        if (m == 0x7fffffff) break;
        for (int a = 0; a < gr; ++a)
            if (p[a] < pe[a] && cC[p[a]] == m) ++p[a];
        ++cnt;
    }
    ntile[g] = (cnt + jt - 1) / jt;
}

// One thread per row group: write the tile headers of its runs.  The group's
// union of P_C columns is cut into runs of jt columns, in ascending column order
// (order 0) or grouped by the set of the group's rows whose P_C row holds the
// column (order 1: row sets in descending bit order, ascending columns inside a
// set).  With order 1 a tile's columns share their output rows, so a row
// multiplies in a tile only where it has outputs; the two orders give the same
// products.  scr (order 1 only): per plan 5 + G arrays of ntiles * jt ints, each
// group using its tiles' range: union columns, row sets and union positions in
// ping-pong pairs, and the C slots of every (column, row) found by the merge.
__global__ void k_group_tiles(int n, int G, int jt, int order, const int *__restrict__ rpC,
                              const int *__restrict__ cC, const int64_t *__restrict__ toff, int64_t ntiles,
                              int *__restrict__ hdr, int *__restrict__ tcols, int *__restrict__ scr)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int ng = (n + G - 1) / G;
    if (g >= ng) return;
    const int hs = G + G * jt;
    int p[kMaxRows], pe[kMaxRows];
    const int i0 = g * G, gr = min(G, n - i0);
    for (int a = 0; a < gr; ++a) {
        p[a] = rpC[i0 + a];
        pe[a] = rpC[i0 + a + 1];
    }
    const int64_t t0 = toff[g], cap = ntiles * jt;
    auto open_tile = [&](int64_t t) {
        int *h = hdr + t * hs;
        for (int a = 0; a < G; ++a) h[a] = (a < gr) ? i0 + a : -1;
        for (int x = 0; x < G * jt; ++x) h[G + x] = -1;
        for (int x = 0; x < jt; ++x) tcols[t * jt + x] = -1;
    };
    if (order == 0) {
        int64_t t = t0;
        int q = 0;
        while (true) {
            int m = 0x7fffffff;
            for (int a = 0; a < gr; ++a)
                if (p[a] < pe[a]) m = min(m, cC[p[a]]);
            if (m == 0x7fffffff) break;
            if (q == 0) open_tile(t);
            int *h = hdr + t * hs;
            tcols[t * jt + q] = m;
            for (int a = 0; a < gr; ++a)
                if (p[a] < pe[a] && cC[p[a]] == m) {
                    h[G + a * jt + q] = p[a];
                    ++p[a];
                }
            if (++q == jt) {
                q = 0;
                ++t;
            }
        }
        return;
    }
    // order 1: union with row sets and slots, then a stable radix sort of the
    // union positions on the row-set bits (least significant first, rows present
    // before rows absent at each bit)
    const int64_t o = t0 * jt;
    int *col = scr + o, *m0 = scr + cap + o, *m1 = scr + 2 * cap + o, *x0 = scr + 3 * cap + o,
        *x1 = scr + 4 * cap + o, *sl = scr + 5 * cap + o * G;
    int cnt = 0;
    while (true) {
        int m = 0x7fffffff;
        for (int a = 0; a < gr; ++a)
            if (p[a] < pe[a]) m = min(m, cC[p[a]]);
        if (m == 0x7fffffff) break;
        int set = 0;
        for (int a = 0; a < G; ++a) {
            int slot = -1;
            if (a < gr && p[a] < pe[a] && cC[p[a]] == m) {
                set |= 1 << a;
                slot = p[a]++;
            }
            sl[(int64_t)cnt * G + a] = slot;
        }
        col[cnt] = m;
        m0[cnt] = set;
        x0[cnt] = cnt;
        ++cnt;
    }
    for (int bit = 0; bit < gr; ++bit) {
        int w = 0;
        for (int x = 0; x < cnt; ++x)
            if ((m0[x] >> bit) & 1) {
                m1[w] = m0[x];
                x1[w++] = x0[x];
            }
        for (int x = 0; x < cnt; ++x)
            if (!((m0[x] >> bit) & 1)) {
                m1[w] = m0[x];
                x1[w++] = x0[x];
            }
        int *tm = m0, *tx = x0;
        m0 = m1;
        x0 = x1;
        m1 = tm;
        x1 = tx;
    }
    for (int x = 0; x < cnt; ++x) {
        const int64_t t = t0 + x / jt;
        const int q = x % jt;
        if (q == 0) open_tile(t);
        int *h = hdr + t * hs;
        const int u = x0[x];
        tcols[t * jt + q] = col[u];
        for (int a = 0; a < gr; ++a) h[G + a * jt + q] = sl[(int64_t)u * G + a];
    }
}

// One thread per (tile, chunk of k): walk the union over the tile's rows of P_A
// (k ascending) for k in [c n / nch, (c + 1) n / nch); keep k when some
// (i_a, k, j) triple exists.  MODE 0 counts entries and triples per (tile,
// chunk), MODE 1 writes the entries; a tile's chunks follow each other, so its
// entries stay in ascending k.  The tile's last chunk writes the padding entry
// that makes the tile's count even (its count includes it, k_pad_counts).  W = 2 (tiles shared by two waves): each entry is two
// halves, one per wave and its jt / 2 columns, each with the A slots of the rows
// that have a live triple in those columns and then those columns' B slots.
template <int MODE>
__global__ void k_tile_entries(int64_t ntiles, int nch, int natoms, int G, int jt, int W, int tr,
                               const int *__restrict__ hdr,
                               const int *__restrict__ tcols, const int *__restrict__ rpA,
                               const int *__restrict__ cA, const int *__restrict__ tmA,
                               const int *__restrict__ rpB, const int *__restrict__ cB,
                               const int *__restrict__ tmB, int64_t *__restrict__ nent,
                               unsigned long long *__restrict__ triples, unsigned long long *__restrict__ rowwork,
                               const int64_t *__restrict__ ebeg, int *__restrict__ ent)
{
    const int64_t tc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tc >= ntiles * nch) return;
    const int64_t t = tc / nch;
    const int c = (int)(tc - t * nch);
    const int k0 = (int)((int64_t)c * natoms / nch), k1 = (int)((int64_t)(c + 1) * natoms / nch);
    const int hs = G + G * jt, es = W * G + jt, jh = jt / W;
    const int *h = hdr + t * hs;
    int pa[kMaxRows], pae[kMaxRows], pb[64], pbe[64], jcol[64];
    // first position in cols[lo, hi) at or past value v
    auto lower = [](const int *__restrict__ cols, int lo, int hi, int v) {
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cols[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    for (int a = 0; a < G; ++a) {
        const int i = h[a];
        pa[a] = (i >= 0) ? lower(cA, rpA[i], rpA[i + 1], k0) : 0;
        pae[a] = (i >= 0) ? lower(cA, pa[a], rpA[i + 1], k1) : 0;
    }
    for (int x = 0; x < jt; ++x) {
        const int j = tcols[t * jt + x];
        jcol[x] = j;
        pb[x] = (j >= 0) ? lower(cB, rpB[j], rpB[j + 1], k0) : 0;
        pbe[x] = (j >= 0) ? lower(cB, pb[x], rpB[j + 1], k1) : 0;
    }
    int64_t w = (MODE == 1) ? ebeg[tc] : 0;
    int64_t cnt = 0;
    unsigned long long tri = 0, rw = 0;
    while (true) {
        int k = 0x7fffffff;
        for (int a = 0; a < G; ++a)
            if (pa[a] < pae[a]) k = min(k, cA[pa[a]]);
        if (k == 0x7fffffff) break;
        int aslot[kMaxRows];
        for (int a = 0; a < G; ++a) {
            aslot[a] = -1;
            if (pa[a] < pae[a] && cA[pa[a]] == k) aslot[a] = tr ? tmA[pa[a]++] : pa[a]++;   // tr: slot of (k, i)
        }
        int bslot[64];
        int ntri = 0;
        for (int x = 0; x < jt; ++x) {
            bslot[x] = -1;
            if (jcol[x] < 0) continue;
            while (pb[x] < pbe[x] && cB[pb[x]] < k) ++pb[x];
            if (pb[x] < pbe[x] && cB[pb[x]] == k) bslot[x] = tr ? pb[x] : tmB[pb[x]];   // (k, j); tr: (j, k)
            if (bslot[x] < 0) continue;
            for (int a = 0; a < G; ++a) ntri += (aslot[a] >= 0 && h[G + a * jt + x] >= 0) ? 1 : 0;
        }
        if (ntri == 0) continue;
        // A row (B column) blocks with no live triple in this entry would only
        // meet zero blocks or outputs outside P_C: drop them, so that the kernels
        // neither copy nor multiply them
        unsigned rowlive[2] = {0u, 0u};
        unsigned long long collive = 0;
        for (int x = 0; x < jt; ++x) {
            if (bslot[x] < 0) continue;
            for (int a = 0; a < G; ++a)
                if (aslot[a] >= 0 && h[G + a * jt + x] >= 0) {
                    rowlive[x / jh] |= 1u << a;
                    collive |= 1ull << x;
                }
        }
        for (int x = 0; x < jt; ++x)
            if (!((collive >> x) & 1ull)) bslot[x] = -1;
        if (MODE == 1) {
            int *e = ent + w * es;
            for (int hf = 0; hf < W; ++hf, e += G + jh) {
                for (int a = 0; a < G; ++a) e[a] = ((rowlive[hf] >> a) & 1u) ? aslot[a] : -1;
                for (int x = 0; x < jh; ++x) e[G + x] = bslot[hf * jh + x];
            }
        }
        ++w;
        ++cnt;
        tri += ntri;
        for (int hf = 0; hf < W; ++hf) rw += __popc(rowlive[hf]);   // rows multiplied
    }
    if (MODE == 1 && c == nch - 1 && w < ebeg[tc + 1]) {   // the padding entry: multiplies nothing
        int *e = ent + w * es;
        for (int x = 0; x < es; ++x) e[x] = -1;
    }
    if (MODE == 0) {
        nent[tc] = cnt;
        atomicAdd(triples, tri);   // integers: order-independent
        atomicAdd(rowwork, rw);
    }
}

// One thread per tile: make the tile's entry count even by counting a padding
// entry in its last chunk.
__global__ void k_pad_counts(int64_t ntiles, int nch, int64_t *__restrict__ nent)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int64_t sum = 0;
    for (int c = 0; c < nch; ++c) sum += nent[t * nch + c];
    if (sum & 1) nent[t * nch + nch - 1] += 1;
}

// One thread per tile: the tile's entry range from the (tile, chunk) ranges.
__global__ void k_tile_ebeg(int64_t ntiles, int nch, const int64_t *__restrict__ ebeg_tc, int64_t *__restrict__ ebeg)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    ebeg[t] = ebeg_tc[t * nch];
}

// One thread per tile of a transposed plan: C slots of (i, j) -> slots of (j, i).
__global__ void k_map_cslots(int64_t ntiles, int G, int jt, const int *__restrict__ tmC, int *__restrict__ hdr)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int *h = hdr + t * (G + G * jt) + G;
    for (int x = 0; x < G * jt; ++x)
        if (h[x] >= 0) h[x] = tmC[h[x]];
}

__global__ __launch_bounds__(1024) void k_scan64(int64_t n, const int64_t *__restrict__ in, int64_t *__restrict__ out)
{
    __shared__ long long part[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    const int64_t chunk = (n + nt - 1) / nt;
    const int64_t lo = min(n, (int64_t)t * chunk), hi = min(n, lo + chunk);
    long long s = 0;
    for (int64_t k = lo; k < hi; ++k) s += in[k];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        long long v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long run = part[t] - s;
    for (int64_t k = lo; k < hi; ++k) {
        out[k] = run;
        run += in[k];
    }
    if (t == nt - 1) out[n] = part[t];
}

__global__ void k_int_to_i64(int n, const int *__restrict__ in, int64_t *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

template <int B, int G, class T = double>
void launch_bg(hipStream_t st, const Plan *plan, const T *A, const T *Bm, double *C, double alpha,
               double beta)
{
    const int64_t nwg = (plan->ntiles + kWaves - 1) / kWaves;
    const int64_t nwg_padded = ((nwg + kXcd - 1) / kXcd) * kXcd;
    k_product_sgpr<B, G, T><<<(unsigned)nwg_padded, 64 * kWaves, 0, st>>>(
        plan->ntiles, nwg_padded, plan->order.as<int>(), plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
        plan->ent.as<int>(), A, Bm, C, alpha, beta);
}

template <int B, int G>
void launch_dpp(hipStream_t st, const Plan *plan, const double *A, const double *Bm, double *C, double alpha,
                double beta, const double *zblk)
{
    const int64_t nwg = (plan->ntiles + kWaves - 1) / kWaves;
    const int64_t nwg_padded = ((nwg + kXcd - 1) / kXcd) * kXcd;
    k_product_f64_dpp<B, G><<<(unsigned)nwg_padded, 64 * kWaves, 0, st>>>(
        plan->ntiles, nwg_padded, plan->order.as<int>(), plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
        plan->ent.as<int>(), A, Bm, zblk, C, alpha, beta);
}

template <int B>
void launch_wg(hipStream_t st, const Plan *plan, const double *A, const double *Bm, double *C, double alpha,
               double beta)
{
    const int64_t nwg_padded = ((plan->ntiles + kXcd - 1) / kXcd) * kXcd;
    k_product_wg<B><<<(unsigned)nwg_padded, 256, 0, st>>>(plan->ntiles, nwg_padded, plan->order.as<int>(),
                                                         plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
                                                         plan->ent.as<int>(), A, Bm, C, alpha, beta);
}

template <int B, int G, int D, class T = double, int W = 1, int TR = 0>
void launch_ring_t(hipStream_t st, const Plan *plan, const T *A, const T *Bm, double *C, double alpha, double beta,
                   const T *zblk, int64_t a_bytes, int64_t b_bytes)
{
    const int64_t nwg_padded = ((plan->ntiles + kXcd - 1) / kXcd) * kXcd;
    // variants 4 and 5: buffer copies when both operands fit a buffer resource; else 64-bit addresses
    const bool buf = (plan->variant == 4 || plan->variant == 5) && a_bytes <= (int64_t)kBufMaxBytes &&
                     b_bytes <= (int64_t)kBufMaxBytes;
    if (buf)
        k_product_ring<B, G, D, T, true, W, TR><<<(unsigned)nwg_padded, 64 * W, 0, st>>>(
            plan->ntiles, nwg_padded, plan->order.as<int>(), plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
            plan->ent.as<int>(), A, Bm, zblk, C, alpha, beta, (unsigned)a_bytes, (unsigned)b_bytes);
    else
        k_product_ring<B, G, D, T, false, W, TR><<<(unsigned)nwg_padded, 64 * W, 0, st>>>(
            plan->ntiles, nwg_padded, plan->order.as<int>(), plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
            plan->ent.as<int>(), A, Bm, zblk, C, alpha, beta, 0u, 0u);
}

// Transposed plans (one-wave tiles of 4 or 8 rows, depth 2) compute C^T = B^T A^T:
// the kernel's A operand is B and its B operand is A.
template <int B, int G, int D, class T = double, int W = 1>
void launch_ring(hipStream_t st, const Plan *plan, const T *A, const T *Bm, double *C, double alpha, double beta,
                 const T *zblk, int64_t a_bytes, int64_t b_bytes)
{
    if constexpr (W == 1 && D == 2 && (G == 4 || G == 8)) {
        if (plan->transposed) {
            launch_ring_t<B, G, D, T, W, 1>(st, plan, Bm, A, C, alpha, beta, zblk, b_bytes, a_bytes);
            return;
        }
    }
    if (plan->transposed) throw Error{BSM_EINVAL, "transposed plan without a transposed kernel"};
    launch_ring_t<B, G, D, T, W, 0>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes);
}

template <int G>
void launch_mfma_f64(hipStream_t st, const Plan *plan, const double *A, const double *Bm, double *C, double alpha,
                     double beta, const double *zblk, int64_t a_bytes, int64_t b_bytes)
{
    const int64_t nwg_padded = ((plan->ntiles + kXcd - 1) / kXcd) * kXcd;
    const bool buf = a_bytes <= (int64_t)kBufMaxBytes && b_bytes <= (int64_t)kBufMaxBytes;
    if (buf)
        k_product_mfma_f64<G, true><<<(unsigned)nwg_padded, 64, 0, st>>>(
            plan->ntiles, nwg_padded, plan->order.as<int>(), plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
            plan->ent.as<int>(), A, Bm, zblk, C, alpha, beta, (unsigned)a_bytes, (unsigned)b_bytes);
    else
        k_product_mfma_f64<G, false><<<(unsigned)nwg_padded, 64, 0, st>>>(
            plan->ntiles, nwg_padded, plan->order.as<int>(), plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
            plan->ent.as<int>(), A, Bm, zblk, C, alpha, beta, 0u, 0u);
}

template <int B>
void launch_b(hipStream_t st, const Plan *plan, const double *A, const double *Bm, double *C, double alpha,
              double beta, const double *zblk, int64_t a_bytes, int64_t b_bytes)
{
    if constexpr (B == 9) {
        if (plan->variant == 6) {   // FP64 matrix cores, direct one-wave plans of 4 or 8 rows
            if (plan->transposed) throw Error{BSM_EINVAL, "variant 6 takes direct plans"};
            switch (plan->G) {
                case 4: launch_mfma_f64<4>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                case 8: launch_mfma_f64<8>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                default: throw Error{BSM_EINVAL, "variant 6 takes 4 or 8 rows per tile"};
            }
        }
    }
    if constexpr (B == 9 || B == 4) {
        if (plan->variant == 5) {   // LDS rings, tiles shared by two waves
            switch (plan->G) {
                case 4: launch_ring<B, 4, 2, double, 2>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                case 8: launch_ring<B, 8, 2, double, 2>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                default: throw Error{BSM_EINVAL, "variant 5 takes 4 or 8 rows per tile"};
            }
        }
        if (plan->variant == 3 || plan->variant == 4) {   // LDS ring, depth 3 or 2
            const bool deep = plan->variant == 3;
            switch (plan->G) {
                case 2: deep ? launch_ring<B, 2, 3>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes)
                             : launch_ring<B, 2, 2>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                case 4: deep ? launch_ring<B, 4, 3>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes)
                             : launch_ring<B, 4, 2>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                case 8: launch_ring<B, 8, 2>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                default: break;
            }
        }
        if (plan->variant == 2) {
            launch_wg<B>(st, plan, A, Bm, C, alpha, beta);
            return;
        }
        if (plan->variant == 1) {
            switch (plan->G) {
                case 2: launch_dpp<B, 2>(st, plan, A, Bm, C, alpha, beta, zblk); return;
                case 4: launch_dpp<B, 4>(st, plan, A, Bm, C, alpha, beta, zblk); return;
                default: break;
            }
        }
    }
    switch (plan->G) {
        case 2: launch_bg<B, 2>(st, plan, A, Bm, C, alpha, beta); break;
        case 4: launch_bg<B, 4>(st, plan, A, Bm, C, alpha, beta); break;
        case 8: launch_bg<B, 8>(st, plan, A, Bm, C, alpha, beta); break;
        default: throw Error{BSM_EINVAL, "rows per wave must be 2, 4 or 8"};
    }
}

template <int B>
void launch_b32(hipStream_t st, const Plan *plan, const float *A, const float *Bm, double *C, double alpha,
                double beta, const float *zblk, int64_t a_bytes, int64_t b_bytes)
{
    if constexpr (B == 9 || B == 4) {
        if (plan->variant == 5) {   // LDS rings, tiles shared by two waves, FP32 operands
            switch (plan->G) {
                case 4: launch_ring<B, 4, 2, float, 2>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                case 8: launch_ring<B, 8, 2, float, 2>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                default: throw Error{BSM_EINVAL, "variant 5 takes 4 or 8 rows per tile"};
            }
        }
        if (plan->variant == 3 || plan->variant == 4) {   // LDS ring, FP32 operands
            switch (plan->G) {
                case 2: launch_ring<B, 2, 2, float>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                case 4: launch_ring<B, 4, 2, float>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                case 8: launch_ring<B, 8, 2, float>(st, plan, A, Bm, C, alpha, beta, zblk, a_bytes, b_bytes); return;
                default: break;
            }
        }
    }
    switch (plan->G) {
        case 2: launch_bg<B, 2, float>(st, plan, A, Bm, C, alpha, beta); break;
        case 4: launch_bg<B, 4, float>(st, plan, A, Bm, C, alpha, beta); break;
        case 8: launch_bg<B, 8, float>(st, plan, A, Bm, C, alpha, beta); break;
        default: throw Error{BSM_EINVAL, "rows per wave must be 2, 4 or 8"};
    }
}

#define BSM_FOR_EACH_B(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

}  // namespace

int default_rows_per_wave(int b) { return b >= 5 ? 4 : (b == 4 ? 4 : 2); }
int default_variant(int b) { return (b == 9 || b == 4) ? 4 : 0; }

void build_plan(Context *ctx, const bsm_pattern_s *PA, const bsm_pattern_s *PB, const bsm_pattern_s *PC,
                Plan *plan, int G, int waves, int transposed)
{
    // transposed: plan D = B^T A^T on P_C (C = D^T); the kernel's A operand is B
    // (rows over P_B, which is symmetric), its B operand is A
    BSM_REQUIRE(!transposed || waves == 1, BSM_EINVAL, "transposed plans use one-wave tiles");
    if (transposed) std::swap(PA, PB);
    hipStream_t st = ctx->stream;
    const int n = PC->natoms, jt = waves * (64 / PC->b);
    BSM_REQUIRE(G == 2 || G == 4 || G == 8 || G == kMaxRows, BSM_EINVAL, "rows per tile must be 2, 4, 8 or 16");
    BSM_REQUIRE(waves == 1 || (waves == 2 && G <= 8), BSM_EINVAL, "two waves per tile take at most 8 rows");
    plan->G = G;
    plan->waves = waves;
    plan->jt = jt;
    const int ng = (n + G - 1) / G;
    const int hs = G + G * jt, es = waves * G + jt;
    DevBuf ntile(ctx, sizeof(int) * ng), ntile64(ctx, sizeof(int64_t) * ng), toff(ctx, sizeof(int64_t) * (ng + 1));
    k_group_union<<<(ng + 127) / 128, 128, 0, st>>>(n, G, PC->rowptr.as<int>(), PC->cols.as<int>(), jt,
                                                    ntile.as<int>());
    k_int_to_i64<<<(ng + 255) / 256, 256, 0, st>>>(ng, ntile.as<int>(), ntile64.as<int64_t>());
    k_scan64<<<1, 1024, 0, st>>>(ng, ntile64.as<int64_t>(), toff.as<int64_t>());
    int64_t nt = 0;
    BSM_HIP_TRY(hipMemcpyAsync(&nt, toff.as<int64_t>() + ng, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    plan->ntiles = nt;
    BSM_REQUIRE(nt < (int64_t)INT32_MAX, BSM_EINVAL, "too many product tiles");
    {
        // launch order: within each span of `span` consecutive row groups, chunk
        // position first, so that the groups' tiles over similar columns run
        // together and share B blocks in L2
        std::vector<int> cnt(ng);
        std::vector<int64_t> off(ng + 1);
        BSM_HIP_TRY(hipMemcpyAsync(cnt.data(), ntile.ptr, sizeof(int) * ng, hipMemcpyDeviceToHost, st));
        BSM_HIP_TRY(hipMemcpyAsync(off.data(), toff.ptr, sizeof(int64_t) * (ng + 1), hipMemcpyDeviceToHost, st));
        BSM_HIP_TRY(hipStreamSynchronize(st));
        std::vector<int> order;
        order.reserve((size_t)nt);
        const int span = std::max(1, ctx->group_span);
        for (int g0 = 0; g0 < ng; g0 += span) {
            const int g1 = std::min(ng, g0 + span);
            int qmax = 0;
            for (int g = g0; g < g1; ++g) qmax = std::max(qmax, cnt[g]);
            for (int q = 0; q < qmax; ++q)
                for (int g = g0; g < g1; ++g)
                    if (q < cnt[g]) order.push_back((int)(off[g] + q));
        }
        plan->order = DevBuf(ctx, sizeof(int) * (size_t)std::max<int64_t>(1, nt));
        if (nt > 0)
            BSM_HIP_TRY(hipMemcpyAsync(plan->order.ptr, order.data(), sizeof(int) * (size_t)nt, hipMemcpyHostToDevice, st));
        BSM_HIP_TRY(hipStreamSynchronize(st));
        plan->span = span;
    }
    plan->hdr = DevBuf(ctx, sizeof(int) * (size_t)std::max<int64_t>(1, nt * hs));
    DevBuf tcols(ctx, sizeof(int) * (size_t)std::max<int64_t>(1, nt * jt));
    {
        const int order = ctx->column_order;
        const size_t scrn = order == 1 ? (size_t)std::max<int64_t>(1, (5 + G) * nt * jt) : 1;
        DevBuf scr(ctx, sizeof(int) * scrn);
        k_group_tiles<<<(ng + 127) / 128, 128, 0, st>>>(n, G, jt, order, PC->rowptr.as<int>(), PC->cols.as<int>(),
                                                        toff.as<int64_t>(), nt, plan->hdr.as<int>(),
                                                        tcols.as<int>(), scr.as<int>());
        BSM_HIP_TRY(hipStreamSynchronize(st));   // before the sort buffers are freed
    }
    // entries are planned per (tile, chunk of k) for parallelism; kPlanChunks chunks per tile
    const int nch = kPlanChunks;
    const int64_t ntc = nt * nch;
    DevBuf nent(ctx, sizeof(int64_t) * (size_t)std::max<int64_t>(1, ntc)), tri(ctx, 2 * sizeof(unsigned long long));
    DevBuf ebeg_tc(ctx, sizeof(int64_t) * (size_t)(ntc + 1));
    plan->ebeg = DevBuf(ctx, sizeof(int64_t) * (size_t)(nt + 1));
    BSM_HIP_TRY(hipMemsetAsync(tri.ptr, 0, 2 * sizeof(unsigned long long), st));
    BSM_HIP_TRY(hipMemsetAsync(plan->ebeg.ptr, 0, sizeof(int64_t) * (size_t)(nt + 1), st));
    int64_t ne = 0;
    unsigned long long ntri[2] = {0, 0};   // triples, rows multiplied
    if (nt > 0) {
        const unsigned grid = (unsigned)((ntc + 127) / 128);
        k_tile_entries<0><<<grid, 128, 0, st>>>(nt, nch, PA->natoms, G, jt, waves, transposed, plan->hdr.as<int>(),
                                                tcols.as<int>(), PA->rowptr.as<int>(), PA->cols.as<int>(),
                                                PA->tmap.as<int>(), PB->rowptr.as<int>(), PB->cols.as<int>(),
                                                PB->tmap.as<int>(), nent.as<int64_t>(),
                                                tri.as<unsigned long long>(), tri.as<unsigned long long>() + 1,
                                                nullptr, nullptr);
        k_pad_counts<<<(unsigned)((nt + 127) / 128), 128, 0, st>>>(nt, nch, nent.as<int64_t>());
        k_scan64<<<1, 1024, 0, st>>>(ntc, nent.as<int64_t>(), ebeg_tc.as<int64_t>());
        k_tile_ebeg<<<(unsigned)((nt + 1 + 127) / 128), 128, 0, st>>>(nt, nch, ebeg_tc.as<int64_t>(),
                                                                      plan->ebeg.as<int64_t>());
        BSM_HIP_TRY(hipMemcpyAsync(&ne, ebeg_tc.as<int64_t>() + ntc, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        BSM_HIP_TRY(hipMemcpyAsync(ntri, tri.ptr, sizeof(ntri), hipMemcpyDeviceToHost, st));
        BSM_HIP_TRY(hipStreamSynchronize(st));
        plan->ent = DevBuf(ctx, sizeof(int) * (size_t)((ne + 4) * es));   // 4 spare entries
        BSM_HIP_TRY(hipMemsetAsync(plan->ent.as<int>() + ne * es, 0xff, sizeof(int) * 4 * es, st));
        k_tile_entries<1><<<grid, 128, 0, st>>>(nt, nch, PA->natoms, G, jt, waves, transposed, plan->hdr.as<int>(),
                                                tcols.as<int>(), PA->rowptr.as<int>(), PA->cols.as<int>(),
                                                PA->tmap.as<int>(), PB->rowptr.as<int>(), PB->cols.as<int>(),
                                                PB->tmap.as<int>(), nullptr, nullptr, nullptr,
                                                ebeg_tc.as<int64_t>(), plan->ent.as<int>());
        BSM_HIP_TRY(hipGetLastError());
    } else {
        plan->ent = DevBuf(ctx, sizeof(int) * 4 * es);
        BSM_HIP_TRY(hipMemsetAsync(plan->ent.ptr, 0xff, sizeof(int) * 4 * es, st));
    }
    BSM_HIP_TRY(hipStreamSynchronize(st));
    plan->nentries = ne;
    plan->triples = (int64_t)ntri[0];
    plan->rowwork = (int64_t)ntri[1];
    plan->flops = 2.0 * (double)PC->b * PC->b * PC->b * (double)ntri[0];
    plan->transposed = transposed;
    if (transposed && nt > 0) {   // outputs go to the slot of (j, i)
        k_map_cslots<<<(unsigned)((nt + 127) / 128), 128, 0, st>>>(nt, G, jt, PC->tmap.as<int>(), plan->hdr.as<int>());
        BSM_HIP_TRY(hipGetLastError());
        BSM_HIP_TRY(hipStreamSynchronize(st));
    }
}

void launch_product_f64(Context *ctx, const Plan *plan, double alpha, const bsm_pattern_s *PA,
                        const double *A, const bsm_pattern_s *PB, const double *Bm, double beta,
                        const bsm_pattern_s *PC, double *C)
{
    if (plan->ntiles == 0) return;
    hipStream_t st = ctx->stream;
    Context::ProfRec rec{plan, nullptr, nullptr, BSM_F64};
    if (ctx->profiling) {
        rec.start = ctx->take_event();
        rec.stop = ctx->take_event();
        BSM_HIP_TRY(hipEventRecord(rec.start, st));
    }
    switch (PC->b) {
#define X(b) \
    case b: launch_b<b>(st, plan, A, Bm, C, alpha, beta, ctx->zero_block.as<double>(), 8 * nelems(PA), 8 * nelems(PB)); break;
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

// A paired launch's 4-row plan, estimated from the class's default plan (about 1.3 times its
// size), fits when free device memory holds twice the estimate and a quarter of the device more.
static bool pair_plan_fits(Context *ctx, const Plan *one)
{
    const double est = 1.3 * (double)(one->ent.bytes + one->hdr.bytes + one->order.bytes + one->ebeg.bytes);
    size_t free_b = 0, total_b = 0;
    BSM_HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    return (double)free_b >= 2.0 * est + std::max(8.0 * (1u << 30), 0.25 * (double)total_b);
}

Plan *get_pair_plan(Context *ctx, const bsm_pattern_s *PA, const bsm_pattern_s *PB, const bsm_pattern_s *PC)
{
    const int b = PC->b;
    if (b != 4 && b != 9) return nullptr;
    if (ctx->product_variant >= 0 && ctx->product_variant != 4) return nullptr;
    // direct 4-row ring plan: 8 rows per paired tile
    auto it = ctx->plans.find(std::make_tuple(PA->id, PB->id, PC->id, 4, 4, 0));
    if (it != ctx->plans.end()) return it->second.get();
    // The 4-row plan is a second plan beside the default one (about 1.3 times its size, 4.9 GB
    // for the 16 A class at 4096 atoms, eight times that at 32768): built only while free
    // device memory holds twice that and a quarter of the device besides (room for what the
    // caller allocates next), else the pair runs as two launches (same results either way)
    if (!pair_plan_fits(ctx, get_plan(ctx, PA, PB, PC))) return nullptr;
    return get_plan_kind(ctx, PA, PB, PC, 4, 4);
}

namespace {
template <int B, int TR>
void launch_pair(hipStream_t st, const Plan *plan, const double *A, const double *A2, const double *Bm, double *C,
                 double *C2, double alpha, double beta, const double *zblk, int64_t a_bytes, int64_t b_bytes)
{
    const int64_t nwg_padded = ((plan->ntiles + kXcd - 1) / kXcd) * kXcd;
    const bool buf = a_bytes <= (int64_t)kBufMaxBytes && b_bytes <= (int64_t)kBufMaxBytes;
    if (buf)
        k_product_ring_pair<B, 8, true, TR><<<(unsigned)nwg_padded, 64, 0, st>>>(
            plan->ntiles, nwg_padded, plan->order.as<int>(), plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
            plan->ent.as<int>(), A, A2, Bm, zblk, C, C2, alpha, beta, (unsigned)a_bytes, (unsigned)a_bytes,
            (unsigned)b_bytes);
    else
        k_product_ring_pair<B, 8, false, TR><<<(unsigned)nwg_padded, 64, 0, st>>>(
            plan->ntiles, nwg_padded, plan->order.as<int>(), plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
            plan->ent.as<int>(), A, A2, Bm, zblk, C, C2, alpha, beta, 0u, 0u, 0u);
}
}  // namespace

void launch_product_pair_f64(Context *ctx, const Plan *plan, double alpha, const bsm_pattern_s *PA,
                             const double *A, const double *A2, const bsm_pattern_s *PB, const double *Bm,
                             double beta, const bsm_pattern_s *PC, double *C, double *C2)
{
    BSM_REQUIRE(plan->variant == 4 && plan->G == 4 && !plan->transposed && (PC->b == 4 || PC->b == 9),
                BSM_EINVAL, "a paired launch takes a direct 4-row ring plan, b = 4 or 9");
    if (plan->ntiles == 0) return;
    hipStream_t st = ctx->stream;
    Context::ProfRec rec{plan, nullptr, nullptr, BSM_F64, 2};
    if (ctx->profiling) {
        rec.start = ctx->take_event();
        rec.stop = ctx->take_event();
        BSM_HIP_TRY(hipEventRecord(rec.start, st));
    }
    const int64_t ab = 8 * nelems(PA), bb = 8 * nelems(PB);
    if (PC->b == 9)
        launch_pair<9, 0>(st, plan, A, A2, Bm, C, C2, alpha, beta, ctx->zero_block.as<double>(), ab, bb);
    else
        launch_pair<4, 0>(st, plan, A, A2, Bm, C, C2, alpha, beta, ctx->zero_block.as<double>(), ab, bb);
    BSM_HIP_TRY(hipGetLastError());
    if (ctx->profiling) {
        BSM_HIP_TRY(hipEventRecord(rec.stop, st));
        ctx->prof.push_back(rec);
    }
}

Plan *get_pair_plan_a(Context *ctx, const bsm_pattern_s *PA, const bsm_pattern_s *PB, const bsm_pattern_s *PC)
{
    const int b = PC->b;
    if (b != 4 && b != 9) return nullptr;
    if (ctx->product_variant >= 0 && ctx->product_variant != 4) return nullptr;
    // transposed 4-row ring plan: the tiles' rows walk B and B2, the shared A is the copied operand
    auto it = ctx->plans.find(std::make_tuple(PA->id, PB->id, PC->id, 4, 4, 2));
    if (it != ctx->plans.end()) return it->second.get();
    if (!pair_plan_fits(ctx, get_plan(ctx, PA, PB, PC))) return nullptr;
    return get_transposed_plan(ctx, PA, PB, PC, 4);
}

void launch_product_pair_a_f64(Context *ctx, const Plan *plan, double alpha, const bsm_pattern_s *PA,
                               const double *A, const bsm_pattern_s *PB, const double *Bm, const double *B2,
                               double beta, const bsm_pattern_s *PC, double *C, double *C2)
{
    BSM_REQUIRE(plan->variant == 4 && plan->G == 4 && plan->transposed && (PC->b == 4 || PC->b == 9),
                BSM_EINVAL, "a paired launch sharing A takes a transposed 4-row ring plan, b = 4 or 9");
    if (plan->ntiles == 0) return;
    hipStream_t st = ctx->stream;
    Context::ProfRec rec{plan, nullptr, nullptr, BSM_F64, 2};
    if (ctx->profiling) {
        rec.start = ctx->take_event();
        rec.stop = ctx->take_event();
        BSM_HIP_TRY(hipEventRecord(rec.start, st));
    }
    // the kernel's row operand is B (and B2), its column operand the shared A
    const int64_t ab = 8 * nelems(PB), bb = 8 * nelems(PA);
    if (PC->b == 9)
        launch_pair<9, 1>(st, plan, Bm, B2, A, C, C2, alpha, beta, ctx->zero_block.as<double>(), ab, bb);
    else
        launch_pair<4, 1>(st, plan, Bm, B2, A, C, C2, alpha, beta, ctx->zero_block.as<double>(), ab, bb);
    BSM_HIP_TRY(hipGetLastError());
    if (ctx->profiling) {
        BSM_HIP_TRY(hipEventRecord(rec.stop, st));
        ctx->prof.push_back(rec);
    }
}

void launch_product_mixed(Context *ctx, const Plan *plan, int prec, double alpha, const bsm_pattern_s *PA,
                          const double *A, const bsm_pattern_s *PB, const double *Bm, double beta,
                          const bsm_pattern_s *PC, double *C)
{
    if (prec == BSM_F64) {
        launch_product_f64(ctx, plan, alpha, PA, A, PB, Bm, beta, PC, C);
        return;
    }
    BSM_REQUIRE(prec == BSM_F32 || prec == BSM_BF16, BSM_EINVAL, "precision must be F64, F32 or BF16");
    if (plan->G > 8) plan = get_plan_kind(ctx, PA, PB, PC, 0, default_rows_per_wave(PC->b));   // wave tiles
    if (plan->variant == 6) plan = get_plan_kind(ctx, PA, PB, PC, 4, plan->G);   // reduced precision: the ring
    // BF16 on the matrix cores for products of two matrices on one pattern (the wide 16 A class,
    // where the dense MFMA tiles pay); the narrower classes run faster on the FP32 VALU ring with
    // BF16-rounded operands, on their own (possibly transposed) plans
    const bool mfma = prec == BSM_BF16 && PC->b == 9 && PA == PB;
    if (mfma && (plan->variant == 5 || plan->transposed))
        plan = get_plan_kind(ctx, PA, PB, PC, 4, plan->G);   // the matrix cores take direct one-wave tiles
    if (plan->ntiles == 0) return;
    hipStream_t st = ctx->stream;
    if (mfma && (plan->G == 4 || plan->G == 8) && (plan->variant == 3 || plan->variant == 4)) {
        // matrix cores: operands packed to BF16 (B transposed), FP32 accumulation
        unsigned short *pa = reinterpret_cast<unsigned short *>(ctx->scratch_f32(0, PA->nnzb * (kPackedBlock / 2)));
        unsigned short *pb = reinterpret_cast<unsigned short *>(ctx->scratch_f32(1, PB->nnzb * (kPackedBlock / 2)));
        k_pack_bf16_blocks<<<(unsigned)((PA->nnzb * kPackedBlock + 255) / 256), 256, 0, st>>>(PA->nnzb, A, pa, 0);
        k_pack_bf16_blocks<<<(unsigned)((PB->nnzb * kPackedBlock + 255) / 256), 256, 0, st>>>(PB->nnzb, Bm, pb, 1);
        Context::ProfRec rec{plan, nullptr, nullptr, prec};
        if (ctx->profiling) {
            rec.start = ctx->take_event();
            rec.stop = ctx->take_event();
            BSM_HIP_TRY(hipEventRecord(rec.start, st));
        }
        const int64_t nwg_padded = ((plan->ntiles + kXcd - 1) / kXcd) * kXcd;
        // variant 4: buffer copies while the packed operands fit a buffer resource
        const int64_t ab = PA->nnzb * (int64_t)kPackedBytes, bb = PB->nnzb * (int64_t)kPackedBytes;
        const bool buf = plan->variant == 4 && ab <= (int64_t)kBufMaxBytes && bb <= (int64_t)kBufMaxBytes;
        auto go = [&](auto kern) {
            kern<<<(unsigned)nwg_padded, 64, 0, st>>>(plan->ntiles, nwg_padded, plan->order.as<int>(),
                                                      plan->hdr.as<int>(), plan->ebeg.as<int64_t>(),
                                                      plan->ent.as<int>(), pa, pb,
                                                      ctx->zero_block.as<unsigned short>(), C, alpha, beta,
                                                      buf ? (unsigned)ab : 0u, buf ? (unsigned)bb : 0u);
        };
        if (plan->G == 8)
            buf ? go(k_product_mfma_bf16<8, true>) : go(k_product_mfma_bf16<8, false>);
        else
            buf ? go(k_product_mfma_bf16<4, true>) : go(k_product_mfma_bf16<4, false>);
        BSM_HIP_TRY(hipGetLastError());
        if (ctx->profiling) {
            BSM_HIP_TRY(hipEventRecord(rec.stop, st));
            ctx->prof.push_back(rec);
        }
        return;
    }
    const int64_t na = nelems(PA), nb = nelems(PB);
    float *a32 = ctx->scratch_f32(0, na), *b32 = ctx->scratch_f32(1, nb);
    const int bf = prec == BSM_BF16 ? 1 : 0;
    k_round_copy<<<(unsigned)((na + 255) / 256), 256, 0, st>>>(na, A, a32, bf);
    k_round_copy<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nb, Bm, b32, bf);
    Context::ProfRec rec{plan, nullptr, nullptr, prec};
    if (ctx->profiling) {
        rec.start = ctx->take_event();
        rec.stop = ctx->take_event();
        BSM_HIP_TRY(hipEventRecord(rec.start, st));
    }
    switch (PC->b) {
#define X(b) \
    case b: launch_b32<b>(st, plan, a32, b32, C, alpha, beta, ctx->zero_block.as<float>(), 4 * na, 4 * nb); break;
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

// Estimated cost of a plan for the ring kernels: rows multiplied plus the
// fixed work of an entry (copies, waits, B reads), worth about 4.5 rows by
// measurement.
static double plan_cost(const Plan *p) { return (double)p->rowwork + 4.5 * (double)p->nentries; }

static std::unique_ptr<Plan> new_plan(Context *ctx, const bsm_pattern_s *A, const bsm_pattern_s *B,
                                      const bsm_pattern_s *C, int variant, int G, int transposed)
{
    std::unique_ptr<Plan> plan(new Plan());
    plan->ids[0] = A->id;
    plan->ids[1] = B->id;
    plan->ids[2] = C->id;
    plan->cutoffs[0] = A->cutoff;
    plan->cutoffs[1] = B->cutoff;
    plan->cutoffs[2] = C->cutoff;
    plan->natoms = C->natoms;
    plan->b = C->b;
    build_plan(ctx, A, B, C, plan.get(), G, variant == 5 ? 2 : 1, transposed);
    plan->variant = variant;
    return plan;
}

Plan *get_transposed_plan(Context *ctx, const bsm_pattern_s *A, const bsm_pattern_s *B, const bsm_pattern_s *C, int G)
{
    auto key = std::make_tuple(A->id, B->id, C->id, 4, G, 2);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) return it->second.get();
    std::unique_ptr<Plan> plan = new_plan(ctx, A, B, C, 4, G, 1);
    Plan *raw = plan.get();
    ctx->plans[key] = std::move(plan);
    return raw;
}

Plan *get_plan_kind(Context *ctx, const bsm_pattern_s *A, const bsm_pattern_s *B, const bsm_pattern_s *C,
                    int variant, int G, bool allow_transposed)
{
    // C = (B^T A^T)^T is an option for the default ring kernel when A and B lie on
    // different patterns (all patterns are symmetric): a wide A times a narrow B
    // then walks the narrow pattern, with far fewer idle lanes
    const bool try_t = allow_transposed && ctx->transposed_plans > 0 && variant == 4 && (G == 4 || G == 8) &&
                       (C->b == 4 || C->b == 9) && A->id != B->id;
    auto key = std::make_tuple(A->id, B->id, C->id, variant, G, try_t ? 1 : 0);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) return it->second.get();
    auto make = [&](int transposed) { return new_plan(ctx, A, B, C, variant, G, transposed); };
    std::unique_ptr<Plan> plan = ctx->transposed_plans == 2 && try_t ? make(1) : make(0);
    if (try_t && ctx->transposed_plans == 1) {
        std::unique_ptr<Plan> alt = make(1);
        if (plan_cost(alt.get()) < plan_cost(plan.get())) plan = std::move(alt);
    }
    Plan *raw = plan.get();
    ctx->plans[key] = std::move(plan);
    return raw;
}

Plan *get_plan(Context *ctx, const bsm_pattern_s *A, const bsm_pattern_s *B, const bsm_pattern_s *C)
{
    int variant = ctx->product_variant >= 0 ? ctx->product_variant : default_variant(C->b);
    if (variant == 6 && C->b != 9) variant = 4;   // the FP64 matrix-core tiles are for b = 9
    if (variant >= 2 && C->b != 9 && C->b != 4) variant = 0;
    int G = variant == 2 ? kMaxRows : (ctx->rows_per_wave > 0 ? ctx->rows_per_wave : default_rows_per_wave(C->b));
    if ((variant == 4 || variant == 5 || variant == 6) && (C->b == 4 || C->b == 9) && ctx->rows_per_wave == 0)
        G = 8;   // measured best for the ring
    if ((variant == 5 || variant == 6) && G < 4) G = 4;   // two-wave and matrix-core tiles take 4 or 8 rows
    return get_plan_kind(ctx, A, B, C, variant, G, true);
}

}  // namespace bsm
