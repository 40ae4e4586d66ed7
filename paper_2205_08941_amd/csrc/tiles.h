// Device code of one product tile (one wavefront), shared by the per-product
// kernels and the persistent batch kernel.  See product.hip for the plan layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

namespace bsm {

// Wave-uniform read-only view: loads through it become scalar loads when the
// address is uniform.
template <class T> using const_as4 = const __attribute__((address_space(4))) T;

// alpha s + beta c with each operation rounded on its own (no fused contraction
// that a compiler may apply one way in one kernel and another way in the next),
// so that every product kernel stores the same bits for the same sums.
__device__ inline double scale_add(double alpha, double s, double beta, double c)
{
    return __dadd_rn(__dmul_rn(alpha, s), __dmul_rn(beta, c));
}

template <int B, int G, class T>
__device__ inline void multiply_entry(const_as4<int> *entu, int64_t q, const_as4<T> *vAu, const T (&bv)[B],
                                      bool bact, const bool (&cact)[G], T (&acc)[G][B])
{
    constexpr int BB = B * B;
    constexpr int ES = G + 64 / B;
#pragma unroll
    for (int a = 0; a < G; ++a) {
        const int as = entu[q * ES + a];
        if (as < 0) continue;
        if (bact && cact[a]) {
            const_as4<T> *ap = vAu + (int64_t)as * BB;
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int m = 0; m < B; ++m) acc[a][r] = fma(ap[r * B + m], bv[m], acc[a][r]);
        }
    }
}

// Tile header, ints: rows[G] (atom ids, -1 = padding), cslot[G][JT] (slot of
// (i_a, j) in C or -1).  Entries of tile t: ebeg[t] .. ebeg[t+1] (an even count;
// an odd list ends in a padding entry whose A slots are all -1), each G + JT
// ints: aslot[G] (slot of (i_a, k) in A or -1), bslot[JT] (slot of (k, j) in B
// or -1).  The entry array has 4 spare entries at its end, so the index
// prefetch past a tile's last entry stays in bounds.
// T = double: FP64 product.  T = float: operands already rounded to FP32 (or to
// BF16 and stored as FP32), FP32 fused multiply-add accumulation in the same
// (k, m) order, the FP32 sums widened to FP64 for alpha, beta and the store.
template <int B, int G, class T>
__device__ inline void tile_sgpr(int64_t tile, const int *__restrict__ hdr, const int64_t *__restrict__ ebeg,
                                 const int *__restrict__ ent, const T *__restrict__ vA, const T *__restrict__ vB,
                                 double *__restrict__ vC, double alpha, double beta)
{
    constexpr int JT = 64 / B;
    constexpr int BB = B * B;
    constexpr int HS = G + G * JT;
    constexpr int ES = G + JT;
    const int lane = threadIdx.x & 63;
    const int jl0 = lane / B, c = lane - jl0 * B;
    const bool lane_ok = jl0 < JT;
    const int jl = lane_ok ? jl0 : JT - 1;     // spare lanes read a valid column and stay masked
    const int *h = hdr + tile * HS;
    int cs[G];
    bool cact[G];
#pragma unroll
    for (int a = 0; a < G; ++a) {
        cs[a] = lane_ok ? h[G + a * JT + jl] : -1;
        cact[a] = cs[a] >= 0;
    }
    T acc[G][B];
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
        for (int r = 0; r < B; ++r) acc[a][r] = T(0);

    const int64_t e0 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile] >> 32)) << 32);
    const int64_t e1 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] >> 32)) << 32);
    const int n = (int)(e1 - e0);                  // even
    const_as4<int> *entu = (const_as4<int> *)(ent + e0 * ES);
    const int *entv = ent + e0 * ES + G + jl;      // this lane's B slot column
    const_as4<T> *vAu = (const_as4<T> *)vA;
    const T *vBc = vB + c;

    // ping-pong buffers: entry q in ba while q+1 loads into bb, then q+1 in bb
    // while q+2 loads into ba; B slot indices run two entries ahead.
    T ba[B], bb[B];
    int ia = entv[0], ib = entv[ES];
    ia = (0 < n) ? ia : -1;
    ib = (1 < n) ? ib : -1;
    {
        const T *bp = vBc + (int64_t)max(ia, 0) * BB;
#pragma unroll
        for (int m = 0; m < B; ++m) ba[m] = bp[m * B];
    }
    for (int q = 0; q < n; q += 2) {
        int ic = entv[(int64_t)(q + 2) * ES];
        ic = (q + 2 < n) ? ic : -1;
        {
            const T *bp = vBc + (int64_t)max(ib, 0) * BB;
#pragma unroll
            for (int m = 0; m < B; ++m) bb[m] = bp[m * B];
        }
        multiply_entry<B, G, T>(entu, q, vAu, ba, ia >= 0, cact, acc);
        int id = entv[(int64_t)(q + 3) * ES];
        id = (q + 3 < n) ? id : -1;
        {
            const T *bp = vBc + (int64_t)max(ic, 0) * BB;
#pragma unroll
            for (int m = 0; m < B; ++m) ba[m] = bp[m * B];
        }
        multiply_entry<B, G, T>(entu, q + 1, vAu, bb, ib >= 0, cact, acc);
        ia = ic;
        ib = id;
    }
#pragma unroll
    for (int a = 0; a < G; ++a) {
        if (!cact[a]) continue;
        double *cp = vC + (int64_t)cs[a] * BB + c;
        if (beta == 0.0) {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * B] = alpha * (double)acc[a][r];
        } else {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * B] = scale_add(alpha, (double)acc[a][r], beta, cp[r * B]);
        }
    }
}

// ---------------------------------------------------------------- DPP variant
// The same tiles and entry lists, with the uniform operand A_{i_a k} held in
// VGPRs instead of SGPRs: lane l of every row of 16 lanes holds elements
// l % 16 + 16 v (v < NA) of the block, loaded with ordinary pipelined vector
// loads, and each FMA takes its A element by a DPP row broadcast
// (row_newbcast: lane n of each 16-lane row to the whole row).  This removes
// the scalar-load round trips of the SGPR variant from the inner loop.
// One output row r of a block product: acc += sum_m A[r][m] * b[m], A[r][m]
// broadcast from lane (r*b + m) % 16 of register (r*b + m) / 16.  The row's
// FMAs form one asm block that starts with two wait states: a VALU write of a
// register followed by a DPP read of it needs them, and the compiler does not
// track that hazard into inline asm.
#define BSM_FMA_DPP(acc, a, bq, lane) "v_fmac_f64_dpp " acc ", " a ", " bq " row_newbcast:" lane " row_mask:0xf bank_mask:0xf\n"

template <int B, int NA, int R, class T = double> struct DppRow;

template <int NA, int R> struct DppRow<9, NA, R, double> {
    static constexpr int e(int m) { return R * 9 + m; }
    __device__ static inline void run(double &acc, const double (&av)[NA], const double (&bv)[9])
    {
        asm("s_nop 1\n"
            BSM_FMA_DPP("%0", "%1", "%10", "%19") BSM_FMA_DPP("%0", "%2", "%11", "%20")
            BSM_FMA_DPP("%0", "%3", "%12", "%21") BSM_FMA_DPP("%0", "%4", "%13", "%22")
            BSM_FMA_DPP("%0", "%5", "%14", "%23") BSM_FMA_DPP("%0", "%6", "%15", "%24")
            BSM_FMA_DPP("%0", "%7", "%16", "%25") BSM_FMA_DPP("%0", "%8", "%17", "%26")
            BSM_FMA_DPP("%0", "%9", "%18", "%27")
            : "+v"(acc)
            : "v"(av[e(0) >> 4]), "v"(av[e(1) >> 4]), "v"(av[e(2) >> 4]), "v"(av[e(3) >> 4]),
              "v"(av[e(4) >> 4]), "v"(av[e(5) >> 4]), "v"(av[e(6) >> 4]), "v"(av[e(7) >> 4]),
              "v"(av[e(8) >> 4]),
              "v"(bv[0]), "v"(bv[1]), "v"(bv[2]), "v"(bv[3]), "v"(bv[4]), "v"(bv[5]), "v"(bv[6]), "v"(bv[7]),
              "v"(bv[8]),
              "n"(e(0) & 15), "n"(e(1) & 15), "n"(e(2) & 15), "n"(e(3) & 15), "n"(e(4) & 15), "n"(e(5) & 15),
              "n"(e(6) & 15), "n"(e(7) & 15), "n"(e(8) & 15));
    }
};

template <int NA, int R> struct DppRow<4, NA, R, double> {
    static constexpr int e(int m) { return R * 4 + m; }
    __device__ static inline void run(double &acc, const double (&av)[NA], const double (&bv)[4])
    {
        asm("s_nop 1\n"
            BSM_FMA_DPP("%0", "%1", "%5", "%9") BSM_FMA_DPP("%0", "%2", "%6", "%10")
            BSM_FMA_DPP("%0", "%3", "%7", "%11") BSM_FMA_DPP("%0", "%4", "%8", "%12")
            : "+v"(acc)
            : "v"(av[e(0) >> 4]), "v"(av[e(1) >> 4]), "v"(av[e(2) >> 4]), "v"(av[e(3) >> 4]),
              "v"(bv[0]), "v"(bv[1]), "v"(bv[2]), "v"(bv[3]),
              "n"(e(0) & 15), "n"(e(1) & 15), "n"(e(2) & 15), "n"(e(3) & 15));
    }
};
#undef BSM_FMA_DPP

// FP32 operands and accumulators: the same rows with v_fmac_f32_dpp (one FP32
// fused multiply-add per element, in m order, as the FP32 reference sums).
#define BSM_FMA_DPP32(acc, a, bq, lane) "v_fmac_f32_dpp " acc ", " a ", " bq " row_newbcast:" lane " row_mask:0xf bank_mask:0xf\n"

template <int NA, int R> struct DppRow<9, NA, R, float> {
    static constexpr int e(int m) { return R * 9 + m; }
    __device__ static inline void run(float &acc, const float (&av)[NA], const float (&bv)[9])
    {
        asm("s_nop 1\n"
            BSM_FMA_DPP32("%0", "%1", "%10", "%19") BSM_FMA_DPP32("%0", "%2", "%11", "%20")
            BSM_FMA_DPP32("%0", "%3", "%12", "%21") BSM_FMA_DPP32("%0", "%4", "%13", "%22")
            BSM_FMA_DPP32("%0", "%5", "%14", "%23") BSM_FMA_DPP32("%0", "%6", "%15", "%24")
            BSM_FMA_DPP32("%0", "%7", "%16", "%25") BSM_FMA_DPP32("%0", "%8", "%17", "%26")
            BSM_FMA_DPP32("%0", "%9", "%18", "%27")
            : "+v"(acc)
            : "v"(av[e(0) >> 4]), "v"(av[e(1) >> 4]), "v"(av[e(2) >> 4]), "v"(av[e(3) >> 4]),
              "v"(av[e(4) >> 4]), "v"(av[e(5) >> 4]), "v"(av[e(6) >> 4]), "v"(av[e(7) >> 4]),
              "v"(av[e(8) >> 4]),
              "v"(bv[0]), "v"(bv[1]), "v"(bv[2]), "v"(bv[3]), "v"(bv[4]), "v"(bv[5]), "v"(bv[6]), "v"(bv[7]),
              "v"(bv[8]),
              "n"(e(0) & 15), "n"(e(1) & 15), "n"(e(2) & 15), "n"(e(3) & 15), "n"(e(4) & 15), "n"(e(5) & 15),
              "n"(e(6) & 15), "n"(e(7) & 15), "n"(e(8) & 15));
    }
};

template <int NA, int R> struct DppRow<4, NA, R, float> {
    static constexpr int e(int m) { return R * 4 + m; }
    __device__ static inline void run(float &acc, const float (&av)[NA], const float (&bv)[4])
    {
        asm("s_nop 1\n"
            BSM_FMA_DPP32("%0", "%1", "%5", "%9") BSM_FMA_DPP32("%0", "%2", "%6", "%10")
            BSM_FMA_DPP32("%0", "%3", "%7", "%11") BSM_FMA_DPP32("%0", "%4", "%8", "%12")
            : "+v"(acc)
            : "v"(av[e(0) >> 4]), "v"(av[e(1) >> 4]), "v"(av[e(2) >> 4]), "v"(av[e(3) >> 4]),
              "v"(bv[0]), "v"(bv[1]), "v"(bv[2]), "v"(bv[3]),
              "n"(e(0) & 15), "n"(e(1) & 15), "n"(e(2) & 15), "n"(e(3) & 15));
    }
};
#undef BSM_FMA_DPP32

template <int B, int NA, class T, int... R>
__device__ inline void fma_block(T (&acc)[B], const T (&av)[NA], const T (&bv)[B], std::integer_sequence<int, R...>)
{
    (DppRow<B, NA, R, T>::run(acc[R], av, bv), ...);
}

// Element l16 + 16 v of the block into register v; indices past the block wrap
// to its start (unused lanes, kept lane-varying so every element arrives by a
// vector load straight into its VGPR).
template <int B, int NA>
__device__ inline void load_a(double (&av)[NA], const double *__restrict__ vA, int slot, int l16)
{
    constexpr int BB = B * B;
    const double *ap = vA + (int64_t)max(slot, 0) * BB;
#pragma unroll
    for (int v = 0; v < NA; ++v) {
        int idx = l16 + 16 * v;
        if (idx >= BB) idx -= BB;
        av[v] = ap[idx];
    }
}

// Lanes whose (k, j) block is absent read a block of zeros instead: the DPP
// broadcast needs every lane of the wave active (a read from an exec-disabled
// source lane is invalid), so absent triples are multiplied by zero rather than
// masked off.
template <int B>
__device__ inline void load_b(double (&bv)[B], const double *__restrict__ vBc, const double *__restrict__ zc, int slot)
{
    const double *bp = (slot >= 0) ? vBc + (int64_t)slot * (B * B) : zc;
#pragma unroll
    for (int m = 0; m < B; ++m) bv[m] = bp[m * B];
}

template <int B, int G, int NA, class T = double>
__device__ inline void dpp_entry(const int (&as)[G], const T (&av)[G][NA], const T (&bv)[B], T (&acc)[G][B])
{
#pragma unroll
    for (int a = 0; a < G; ++a) {
        if (as[a] < 0) continue;   // wave-uniform
        fma_block<B, NA, T>(acc[a], av[a], bv, std::make_integer_sequence<int, B>{});
    }
}

template <int B, int G>
__device__ inline void tile_dpp(int64_t tile, const int *__restrict__ hdr, const int64_t *__restrict__ ebeg,
                                const int *__restrict__ ent, const double *__restrict__ vA,
                                const double *__restrict__ vB, const double *__restrict__ zblk,
                                double *__restrict__ vC, double alpha, double beta)
{
    constexpr int JT = 64 / B;
    constexpr int BB = B * B;
    constexpr int NA = (BB + 15) / 16;
    constexpr int HS = G + G * JT;
    constexpr int ES = G + JT;
    const int lane = threadIdx.x & 63;
    const int l16 = lane & 15;
    const int jl0 = lane / B, c = lane - jl0 * B;
    const bool lane_ok = jl0 < JT;
    const int jl = lane_ok ? jl0 : JT - 1;
    const int *h = hdr + tile * HS;
    int cs[G];
    bool cact[G];
#pragma unroll
    for (int a = 0; a < G; ++a) {
        cs[a] = lane_ok ? h[G + a * JT + jl] : -1;
        cact[a] = cs[a] >= 0;
    }
    double acc[G][B];
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
        for (int r = 0; r < B; ++r) acc[a][r] = 0.0;

    const int64_t e0 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile] >> 32)) << 32);
    const int64_t e1 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] >> 32)) << 32);
    const int n = (int)(e1 - e0);                  // even
    const_as4<int> *entu = (const_as4<int> *)(ent + e0 * ES);
    const int *entv = ent + e0 * ES + G + jl;
    const double *vBc = vB + c;
    const double *zc = zblk + c;

    // ping-pong: entry q in (xa, ba) while q+1 loads into (xb, bb), and so on;
    // B slot indices two entries ahead, A slots are wave-uniform scalar loads.
    double xa[G][NA], xb[G][NA], ba[B], bb[B];
    int asa[G], asb[G];
    int ia = entv[0], ib = entv[ES];
    ia = (0 < n) ? ia : -1;
    ib = (1 < n) ? ib : -1;
#pragma unroll
    for (int a = 0; a < G; ++a) {
        asa[a] = (0 < n) ? entu[a] : -1;
        load_a<B, NA>(xa[a], vA, asa[a], l16);
    }
    load_b<B>(ba, vBc, zc, ia);
    for (int q = 0; q < n; q += 2) {
        int ic = entv[(int64_t)(q + 2) * ES];
        ic = (q + 2 < n) ? ic : -1;
#pragma unroll
        for (int a = 0; a < G; ++a) {
            asb[a] = entu[(int64_t)(q + 1) * ES + a];
            load_a<B, NA>(xb[a], vA, asb[a], l16);
        }
        load_b<B>(bb, vBc, zc, ib);
        dpp_entry<B, G, NA>(asa, xa, ba, acc);
        int id = entv[(int64_t)(q + 3) * ES];
        id = (q + 3 < n) ? id : -1;
#pragma unroll
        for (int a = 0; a < G; ++a) {
            asa[a] = (q + 2 < n) ? entu[(int64_t)(q + 2) * ES + a] : -1;
            load_a<B, NA>(xa[a], vA, asa[a], l16);
        }
        load_b<B>(ba, vBc, zc, ic);
        dpp_entry<B, G, NA>(asb, xb, bb, acc);
        ia = ic;
        ib = id;
    }
#pragma unroll
    for (int a = 0; a < G; ++a) {
        if (!cact[a]) continue;
        double *cp = vC + (int64_t)cs[a] * BB + c;
        if (beta == 0.0) {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * B] = alpha * acc[a][r];
        } else {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * B] = scale_add(alpha, acc[a][r], beta, cp[r * B]);
        }
    }
}

// ---------------------------------------------------------------- workgroup tiles
// One tile of 16 rows x JT columns per workgroup of 4 wavefronts; wave w owns
// rows 4w .. 4w+3 with the lane layout of tile_dpp.  All four waves read the
// same B_kj blocks, so the workgroup stages them in LDS, two entries at a time
// (double-buffered: the next pair is fetched from global memory into
// registers while the current pair is multiplied, then written to the other
// buffer; one barrier per pair).  Absent (k, j) blocks are staged as zeros.  A
// blocks belong to single waves and are loaded as in tile_dpp.  An entry in
// which none of a wave's rows has an A block costs that wave no FMAs.
template <int B> struct WgTile {
    static constexpr int kJT = 64 / B, kBB = B * B;
    static constexpr int kStage = 2 * kJT * kBB;   // doubles per LDS buffer (two entries)
};

template <int B>
__device__ inline void tile_wg(int64_t tile, const int *__restrict__ hdr, const int64_t *__restrict__ ebeg,
                               const int *__restrict__ ent, const double *__restrict__ vA,
                               const double *__restrict__ vB, double *__restrict__ vC, double alpha, double beta,
                               double *__restrict__ lds)
{
    constexpr int JT = WgTile<B>::kJT, BB = WgTile<B>::kBB, STAGE = WgTile<B>::kStage;
    constexpr int NA = (BB + 15) / 16;
    constexpr int G = 16, GW = 4;                 // rows per tile, rows per wave
    constexpr int HS = G + G * JT, ES = G + JT;
    constexpr int U = (STAGE + 255) / 256;        // staged doubles per thread
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, l16 = lane & 15;
    const int jl0 = lane / B, c = lane - jl0 * B;
    const bool lane_ok = jl0 < JT;
    const int jl = lane_ok ? jl0 : JT - 1;
    const int *h = hdr + tile * HS;
    int cs[GW];
    bool cact[GW];
#pragma unroll
    for (int a = 0; a < GW; ++a) {
        cs[a] = lane_ok ? h[G + (GW * w + a) * JT + jl] : -1;
        cact[a] = cs[a] >= 0;
    }
    double acc[GW][B];
#pragma unroll
    for (int a = 0; a < GW; ++a)
#pragma unroll
        for (int r = 0; r < B; ++r) acc[a][r] = 0.0;

    const int64_t e0 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile] >> 32)) << 32);
    const int64_t e1 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] >> 32)) << 32);
    const int n = (int)(e1 - e0);                  // even
    const int *entg = ent + e0 * ES;
    const_as4<int> *entu = (const_as4<int> *)entg;

    // Staging pipeline over pairs of entries (stages): the B slots of stage
    // s + 2 and the B values of stage s + 1 are loaded while stage s is
    // multiplied, so neither the slot nor the value load stalls the barrier.
    // Thread tid stages doubles tid + 256 u of a stage.
    int sl[U], sl2[U];
    double pf[U];
    auto fetch_slots = [&](int (&dst)[U], int q) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = tid + 256 * u;
            dst[u] = -1;
            if (idx < STAGE) {
                const int e = idx / (JT * BB), col = (idx - e * (JT * BB)) / BB;
                if (q + e < n) dst[u] = entg[(int64_t)(q + e) * ES + G + col];
            }
        }
    };
    auto fetch_values = [&](const int (&src)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = tid + 256 * u;
            const int el = (idx % (JT * BB)) % BB;
            pf[u] = src[u] >= 0 ? vB[(int64_t)src[u] * BB + el] : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = tid + 256 * u;
            if (idx < STAGE) lds[buf * STAGE + idx] = pf[u];
        }
    };
    auto read_b = [&](double (&bv)[B], int buf, int e) {
        const double *p = lds + buf * STAGE + e * (JT * BB) + jl * BB + c;
#pragma unroll
        for (int m = 0; m < B; ++m) bv[m] = p[m * B];
    };
    // A blocks of one entry for this wave's rows (rows without a block load nothing)
    auto load_rows = [&](double (&x)[GW][NA], int (&as)[GW], int q) {
#pragma unroll
        for (int a = 0; a < GW; ++a) {
            as[a] = q < n ? entu[(int64_t)q * ES + GW * w + a] : -1;
            if (as[a] >= 0) load_a<B, NA>(x[a], vA, as[a], l16);
        }
    };

    double xa[GW][NA], xb[GW][NA], bv[B];
    int asa[GW], asb[GW];
    fetch_slots(sl, 0);
    fetch_values(sl);
    store(0);
    fetch_slots(sl, 2);
    load_rows(xa, asa, 0);
    __syncthreads();
    for (int q = 0; q < n; q += 2) {
        const int buf = (q >> 1) & 1;
        const bool more = q + 2 < n;
        if (more) {
            fetch_values(sl);            // stage q + 2
            fetch_slots(sl2, q + 4);     // stage q + 4
        }
        load_rows(xb, asb, q + 1);
        read_b(bv, buf, 0);
        dpp_entry<B, GW, NA>(asa, xa, bv, acc);
        load_rows(xa, asa, q + 2);
        read_b(bv, buf, 1);
        dpp_entry<B, GW, NA>(asb, xb, bv, acc);
        if (more) {
            store(buf ^ 1);
#pragma unroll
            for (int u = 0; u < U; ++u) sl[u] = sl2[u];
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < GW; ++a) {
        if (!cact[a]) continue;
        double *cp = vC + (int64_t)cs[a] * BB + c;
        if (beta == 0.0) {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * B] = alpha * acc[a][r];
        } else {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * B] = scale_add(alpha, acc[a][r], beta, cp[r * B]);
        }
    }
}

// ---------------------------------------------------------------- LDS-ring wave tiles
// The tiles and lane layout of tile_dpp, with both operands of an entry copied
// from global memory straight into a per-wave LDS ring of D entries by
// asynchronous LDS-DMA loads (4 bytes per lane, contiguous in lane order).
// Data in flight occupies no VGPRs, so D - 1 entries are fetched ahead of the
// multiply.  Every block of every entry is copied by the same number of DMA
// instructions, reading the zero block for an absent A_{i_a k} or B_kj, so the
// number of loads issued after an entry is known and one s_waitcnt per entry
// (vmcnt at most that number, clamped to the counter's 63) orders it before
// its LDS reads.  Block slot indices come through the scalar cache, so no
// other vector loads share the vmcnt counter in the loop.
template <int B, int G, class T = double> struct RingEntry {
    static constexpr int kBlocks = G + 64 / B;               // A rows, then B columns
    static constexpr int kBytes = kBlocks * B * B * (int)sizeof(T);
    static constexpr int kDwords = B * B * (int)sizeof(T) / 4;   // per block
    static constexpr int kInstPerBlock = (kDwords + 63) / 64;
    static constexpr int kInst = kBlocks * kInstPerBlock;    // DMA loads per entry
};

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(3))) char lds_char_t;
template <class T> using lds_const_t = const __attribute__((address_space(3))) T;

// s_waitcnt with vmcnt <= vm (expcnt and lgkmcnt not waited on)
template <int VM> __device__ inline void wait_vmcnt()
{
    static_assert(VM >= 0 && VM <= 63, "vmcnt is 6 bits");
    __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Instruction I of a block's DMA copies dwords s_I + lane with s_I = 64 I,
// except that the last instruction of a block longer than 64 dwords starts at
// DW - 64: every lane copies (dwords below 64 I are copied twice, with the same
// values), so no lane mask and no branch is needed.  A block shorter than 64
// dwords is copied by the lanes below DW.  The immediate offset 4 s_I moves
// both the global and the LDS address.
template <int IPB, int DW, int... I>
__device__ inline void dma_block(const char *g, lds_void_t *l, int lane, std::integer_sequence<int, I...>)
{
    if constexpr (DW >= 64) {
        (__builtin_amdgcn_global_load_lds((const void *)g, l, 4, 4 * (I < IPB - 1 ? 64 * I : DW - 64), 0), ...);
    } else {
        static_assert(IPB == 1, "one instruction per short block");
        if (lane < DW) __builtin_amdgcn_global_load_lds((const void *)g, l, 4, 0, 0);
    }
}

// The same copy through a raw buffer resource: voffset = the block's byte
// offset + 4 lane.  An absent block (slot -1) has offset 2^32 - block bytes:
// with the lane and immediate offsets it stays below 2^32 and above the
// resource's size, so the range check returns zeros for every lane (no zero
// block, no select).
template <int IPB, int DW, int... I>
__device__ inline void dma_block_buf(__amdgpu_buffer_rsrc_t rs, unsigned vo, lds_void_t *l, int lane,
                                     std::integer_sequence<int, I...>)
{
    if constexpr (DW >= 64) {
        (__builtin_amdgcn_raw_ptr_buffer_load_lds(rs, l, 4, vo, 0, 4 * (I < IPB - 1 ? 64 * I : DW - 64), 0), ...);
    } else {
        static_assert(IPB == 1, "one instruction per short block");
        if (lane < DW) __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, l, 4, vo, 0, 0, 0);
    }
}

// Largest operand (bytes) the buffer copies address: absent-block offsets
// (2^32 - block bytes and up) must lie past it.
constexpr unsigned kBufMaxBytes = 0xfffff000u;

// T = double: FP64 product.  T = float: operands already rounded (FP32, or BF16
// stored as FP32), FP32 fused multiply-adds in the same (k, m) order, the sums
// widened to FP64 for alpha, beta and the store.
// BUF: copies through raw buffer resources over A and B (a_bytes, b_bytes, each
// at most kBufMaxBytes): one scalar multiply and one vector add per block
// instead of 64-bit address arithmetic and a zero-block select.
// W = 2: the tile has 2 JT columns and two waves of one workgroup share it,
// wave w taking columns w JT .. w JT + JT - 1 with its own ring.  Both waves walk
// the tile's one list of k; each entry holds a half per wave (A slots of the
// rows with outputs in that wave's columns, then its B slots), and a barrier per
// step keeps the two waves on the same entry, so that the A blocks both copy
// are fetched from HBM once and found in cache by the other wave.
// TR = 1: the tile computes D = B^T A^T on P_C for C = D^T (the launch passes
// the operands swapped, the plan holds their slots): every block is read
// transposed from the ring and the result is stored transposed, at the slot of
// (j, i) that the plan's header gives.  Each element sums the same terms in the
// same order as the direct product.
// DU = 2: two products that share B and the patterns, C = A B and C2 = A2 B, on
// one plan of G / 2 rows: the tile's first G / 2 rows multiply A's blocks, the
// other G / 2 the same slots of A2, and every B block copied serves both (with
// TR = 1 on a transposed plan: C = (B^T A^T)^T and C2 = (B^T A2^T)^T, i.e. two
// products sharing their left operand).  Each product's elements sum the same
// terms in the same order as its own launch.
template <int B, int G, int D, class T = double, bool BUF = false, int W = 1, int TR = 0, int DU = 1>
__device__ __attribute__((always_inline)) inline void tile_ring(int64_t tile, const int *__restrict__ hdr, const int64_t *__restrict__ ebeg,
                                 const int *__restrict__ ent, const T *__restrict__ vA, const T *__restrict__ vB,
                                 const T *__restrict__ zblk, double *__restrict__ vC, double alpha, double beta,
                                 lds_char_t *ring, unsigned a_bytes = 0, unsigned b_bytes = 0,
                                 const T *__restrict__ vA2 = nullptr, double *__restrict__ vC2 = nullptr,
                                 unsigned a2_bytes = 0)
{
    using RE = RingEntry<B, G, T>;
    static_assert(W == 1 || W == 2, "one or two waves per tile");
    static_assert(TR == 0 || W == 1, "transposed products use one-wave tiles");
    static_assert(DU == 1 || (DU == 2 && W == 1 && G % 2 == 0), "paired products: one-wave tiles");
    constexpr int ESZ = (int)sizeof(T);
    constexpr int JT = 64 / B;
    constexpr int BB = B * B;
    constexpr int NA = (BB + 15) / 16;
    constexpr int GP = G / DU;                 // rows of the plan
    constexpr int HS = GP + GP * JT * W;
    constexpr int ES = (GP + JT) * W;
    constexpr int NS = GP + JT;                // plan slots per entry and wave
    constexpr int NB = RE::kBlocks, DW = RE::kDwords, IPB = RE::kInstPerBlock, NI = RE::kInst;
    const int lane = threadIdx.x & 63;
    const int w = W > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
    const int l16 = lane & 15;
    const int jl0 = lane / B, c = lane - jl0 * B;
    const bool lane_ok = jl0 < JT;
    const int jl = lane_ok ? jl0 : JT - 1;
    const int *h = hdr + tile * HS;
    int cs[G];
    bool cact[G];
#pragma unroll
    for (int a = 0; a < G; ++a) {
        cs[a] = lane_ok ? h[GP + (a % GP) * JT * W + w * JT + jl] : -1;
        cact[a] = cs[a] >= 0;
    }
    T acc[G][B];
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
        for (int r = 0; r < B; ++r) acc[a][r] = T(0);

    const int64_t e0 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile] >> 32)) << 32);
    const int64_t e1 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] >> 32)) << 32);
    const int n = (int)(e1 - e0);
    const_as4<int> *entu = (const_as4<int> *)(ent + e0 * ES + w * NS);

    // Copy an entry, given its slots, into ring position P; keep its A slots in
    // `asl`.  The DMA's immediate offset advances the global and the LDS address
    // together.  The slots of the entry copied next are loaded (scalar loads)
    // before the current copies are issued, so their latency overlaps them; near
    // the tile's end these loads read the next tile's entries or the plan's four
    // spare entries, which are not used.
    const int lane4 = 4 * lane;
    auto load_slots = [&](int q, int (&sl)[NS]) {
#pragma unroll
        for (int blk = 0; blk < NS; ++blk) sl[blk] = entu[(int64_t)q * ES + blk];
    };
    const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc((void *)vA, 0, (int)a_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc((void *)vB, 0, (int)b_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsA2 =
        __builtin_amdgcn_make_buffer_rsrc((void *)(DU == 2 ? vA2 : vA), 0, (int)(DU == 2 ? a2_bytes : a_bytes), 0x00020000);
    // ring block blk: A rows (the plan's rows, then for DU = 2 the same slots of A2), then B columns
    auto issue = [&](auto P, const int (&sl)[NS], int (&asl)[G]) {
        lds_char_t *slot = ring + decltype(P)::value * RE::kBytes;
#pragma unroll
        for (int a = 0; a < G; ++a) asl[a] = sl[a % GP];
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) {
            lds_void_t *l = (lds_void_t *)(slot + blk * (BB * ESZ));
            const int s_ = blk < G ? sl[blk % GP] : sl[GP + (blk - G)];
            if constexpr (BUF) {
                const unsigned vo = (unsigned)s_ * (unsigned)(BB * ESZ) + (unsigned)lane4;
                dma_block_buf<IPB, DW>(blk < GP ? rsA : (blk < G ? rsA2 : rsB), vo, l, lane,
                                       std::make_integer_sequence<int, IPB>{});
            } else {
                // absent blocks (slot -1) copy the zero block; selected with masks, not a branch
                const T *base = blk < GP ? vA : (blk < G ? (DU == 2 ? vA2 : vA) : vB);
                const uint64_t real = (uint64_t)base + (uint64_t)((int64_t)s_ * (BB * ESZ));
                const uint64_t neg = (uint64_t)(int64_t)(s_ >> 31);
                const char *g = reinterpret_cast<const char *>((real & ~neg) | ((uint64_t)zblk & neg)) + lane4;
                dma_block<IPB, DW>(g, l, lane, std::make_integer_sequence<int, IPB>{});
            }
        }
    };
    // at most `later` entries' copies still in flight
    auto wait_for = [&](auto L) {
        constexpr int later = decltype(L)::value;
        wait_vmcnt<(later * NI < 63 ? later * NI : 63)>();
    };
    // multiply the entry held at ring position P
    auto compute = [&](auto P, const int (&as)[G]) {
        const lds_char_t *slot = ring + decltype(P)::value * RE::kBytes;
        T bv[B];
        lds_const_t<T> *bp = (lds_const_t<T> *)(slot + (G + jl) * (BB * ESZ)) + (TR ? c * B : c);
#pragma unroll
        for (int m = 0; m < B; ++m) bv[m] = bp[TR ? m : m * B];   // element (m, c) of the B operand
        auto read_row = [&](T (&xr)[NA], int a) {
            lds_const_t<T> *ap = (lds_const_t<T> *)(slot + a * (BB * ESZ));
#pragma unroll
            for (int v = 0; v < NA; ++v) {
                int idx = l16 + 16 * v;
                if (idx >= BB) idx -= BB;
                if constexpr (TR) idx = (idx % B) * B + idx / B;   // element (r, m) of the A operand
                xr[v] = ap[idx];
            }
        };
        if constexpr (G <= 4) {
            // all rows' A values read up front (their LDS latency overlaps)
            T xa[G][NA];
#pragma unroll
            for (int a = 0; a < G; ++a)
                if (as[a] >= 0) read_row(xa[a], a);
            dpp_entry<B, G, NA, T>(as, xa, bv, acc);
        } else {
            // two rows of A live next to 8 rows of sums: row a + 1 is read while
            // row a is multiplied (a row without A reads a block it does not use)
            T xr[2][NA];
            read_row(xr[0], 0);
#pragma unroll
            for (int a = 0; a < G; ++a) {
                if (a + 1 < G) read_row(xr[(a + 1) & 1], a + 1);
                if (as[a] >= 0) fma_block<B, NA, T>(acc[a], xr[a & 1], bv, std::make_integer_sequence<int, B>{});
            }
        }
    };
    static_assert(D >= 2 && D <= 3, "ring depth 2 or 3");

    // Every step copies the entry D - 1 ahead, also past the tile's end (the
    // next tile's entries or the plan's spare entries: in bounds, never
    // multiplied), so the steps are straight-line code and each waits for the
    // same count; the tile ends by draining its copies.  sbuf[p] holds the slots
    // of the entry copied next into ring position p; they are loaded one step
    // ahead, up to D entries past the tile.  Entry counts are even, so for D = 2
    // both steps of an iteration are inside the tile.
    int asl[D][G];
    int sbuf[D][NS];
    if (n > 0) {
        load_slots(0, sbuf[0]);
        load_slots(1, sbuf[1]);
        issue(std::integral_constant<int, 0>{}, sbuf[0], asl[0]);
        if constexpr (D == 3) {
            load_slots(2, sbuf[2]);
            issue(std::integral_constant<int, 1>{}, sbuf[1], asl[1]);
        }
    }
    for (int q0 = 0; q0 < n; q0 += D) {
        // ring position of entry q0 + r is r; entry q0 + r + D - 1 goes to (r + D - 1) % D
        auto step = [&](auto R) {
            constexpr int r = decltype(R)::value;
            constexpr int pn = (r + D - 1) % D;
            if constexpr (D == 3)
                if (q0 + r >= n) return;
            if constexpr (W > 1) __builtin_amdgcn_s_barrier();   // both waves at entry q0 + r
            load_slots(q0 + r + D, sbuf[r]);   // entry q0 + r's slots are no longer needed
            __builtin_amdgcn_sched_barrier(0);    // these loads first: their latency overlaps the copies
            issue(std::integral_constant<int, pn>{}, sbuf[pn], asl[pn]);
            wait_for(std::integral_constant<int, D - 1>{});
            compute(std::integral_constant<int, r>{}, asl[r]);
        };
        step(std::integral_constant<int, 0>{});
        step(std::integral_constant<int, 1>{});
        if constexpr (D == 3) step(std::integral_constant<int, 2>{});
    }
    wait_vmcnt<0>();
#pragma unroll
    for (int a = 0; a < G; ++a) {
        if (!cact[a]) continue;
        // TR: element (r, c) of D is element (c, r) of C's block
        double *cp = (DU == 2 && a >= GP ? vC2 : vC) + (int64_t)cs[a] * BB + (TR ? c * B : c);
        constexpr int RS = TR ? 1 : B;
        if (beta == 0.0) {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * RS] = alpha * (double)acc[a][r];
        } else {
#pragma unroll
            for (int r = 0; r < B; ++r) cp[r * RS] = scale_add(alpha, (double)acc[a][r], beta, cp[r * RS]);
        }
    }
}

// ---------------------------------------------------------------- FP64 matrix-core tiles (b = 9)
// The ring tiles' FP64 product on the matrix cores (v_mfma_f64_16x16x4_f64), kept
// as a measured alternative to the VALU tile: the same plan (G = 4 or 8 rows x 7
// columns), the same two-slot LDS ring of FP64 blocks as stored, one entry ahead.
// The tile's 9 G output rows are ceil(9 G / 16) MFMA row tiles, its 63 columns 4
// column tiles; an entry's 9-long contraction is three K = 4 steps (12, the last 3
// zero).  A lane's operands of step s are element (r, 4 s + g) of the A rows and
// (4 s + g, c) of the B columns (r, c: its row and column within the row and column
// tile, g = lane / 16); a row tile whose rows all lack an A block in the entry is
// skipped.  The matrix core multiplies every block pair of a row tile, absent B
// blocks (staged from the zero block) included: dense 16 x 16 tiles over the
// lens-shaped triple set.  Sums are FP64, in the matrix core's order.
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <int G, bool BUF = false>
__device__ __attribute__((always_inline)) inline void tile_mfma_f64(
    int64_t tile, const int *__restrict__ hdr, const int64_t *__restrict__ ebeg, const int *__restrict__ ent,
    const double *__restrict__ vA, const double *__restrict__ vB, const double *__restrict__ zblk,
    double *__restrict__ vC, double alpha, double beta, lds_char_t *ring, unsigned a_bytes = 0,
    unsigned b_bytes = 0)
{
    using RE = RingEntry<9, G, double>;
    constexpr int B = 9, JT = 7, BB = 81, D = 2;
    constexpr int ROWS = 9 * G, RT = (ROWS + 15) / 16;
    constexpr int HS = G + G * JT, ES = G + JT;
    constexpr int NB = RE::kBlocks, DW = RE::kDwords, IPB = RE::kInstPerBlock, NI = RE::kInst;
    static_assert(NB == ES, "one ring block per entry slot");
    const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
    const int *h = hdr + tile * HS;

    const int64_t e0 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile] >> 32)) << 32);
    const int64_t e1 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] >> 32)) << 32);
    const int n = (int)(e1 - e0);   // even
    const_as4<int> *entu = (const_as4<int> *)(ent + e0 * ES);

    // element offsets (doubles) of this lane's operand rows / columns inside a slot, -1: padding
    int aoff[RT], boff[4];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int r = 16 * t + l16;
        aoff[t] = r < ROWS ? (r / 9) * BB + (r % 9) * B : -1;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int cc = 16 * u + l16;
        boff[u] = cc < 63 ? (G + cc / 9) * BB + cc % 9 : -1;
    }
    f64x4_t acc[RT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[t][u] = f64x4_t{0.0, 0.0, 0.0, 0.0};

    const int lane4 = 4 * lane;
    auto load_slots = [&](int q, int (&sl)[NB]) {
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) sl[blk] = entu[(int64_t)q * ES + blk];
    };
    const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc((void *)vA, 0, (int)a_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc((void *)vB, 0, (int)b_bytes, 0x00020000);
    auto issue = [&](auto P, const int (&sl)[NB], int (&asl)[G]) {
        lds_char_t *slot = ring + decltype(P)::value * RE::kBytes;
#pragma unroll
        for (int a = 0; a < G; ++a) asl[a] = sl[a];
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) {
            lds_void_t *l = (lds_void_t *)(slot + blk * (BB * 8));
            if constexpr (BUF) {
                const unsigned vo = (unsigned)sl[blk] * (unsigned)(BB * 8) + (unsigned)lane4;
                dma_block_buf<IPB, DW>(blk < G ? rsA : rsB, vo, l, lane, std::make_integer_sequence<int, IPB>{});
            } else {
                const uint64_t real = (uint64_t)(blk < G ? vA : vB) + (uint64_t)((int64_t)sl[blk] * (BB * 8));
                const uint64_t neg = (uint64_t)(int64_t)(sl[blk] >> 31);
                const char *gp = reinterpret_cast<const char *>((real & ~neg) | ((uint64_t)zblk & neg)) + lane4;
                dma_block<IPB, DW>(gp, l, lane, std::make_integer_sequence<int, IPB>{});
            }
        }
    };
    auto compute = [&](auto P, const int (&as)[G]) {
        lds_const_t<double> *slot = (lds_const_t<double> *)(ring + decltype(P)::value * RE::kBytes);
        bool tact[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            bool any = false;
#pragma unroll
            for (int a = 0; a < G; ++a)
                if (9 * a < 16 * t + 16 && 9 * a + 9 > 16 * t) any |= as[a] >= 0;
            tact[t] = any;
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int k = 4 * s + g;
            const bool kok = k < B;
            double av[RT], bv[4];
            // padding rows / columns and k >= 9 read element 0 of the slot and use 0
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const bool ok = kok && aoff[t] >= 0;
                const double v = slot[ok ? aoff[t] + k : 0];
                av[t] = ok ? v : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool ok = kok && boff[u] >= 0;
                const double v = slot[ok ? boff[u] + k * B : 0];
                bv[u] = ok ? v : 0.0;
            }
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                if (!tact[t]) continue;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[u], acc[t][u], 0, 0, 0);
            }
        }
    };

    // two ring positions; each step copies the entry one ahead (past the tile's end:
    // the next tile's entries or the plan's spare entries, in bounds, never multiplied)
    int asl[D][G];
    int sbuf[D][NB];
    if (n > 0) {
        load_slots(0, sbuf[0]);
        load_slots(1, sbuf[1]);
        issue(std::integral_constant<int, 0>{}, sbuf[0], asl[0]);
    }
    for (int q0 = 0; q0 < n; q0 += D) {
        auto step = [&](auto R) {
            constexpr int r = decltype(R)::value;
            constexpr int pn = (r + 1) % D;
            load_slots(q0 + r + D, sbuf[r]);
            __builtin_amdgcn_sched_barrier(0);
            issue(std::integral_constant<int, pn>{}, sbuf[pn], asl[pn]);
            wait_vmcnt<NI < 63 ? NI : 63>();
            compute(std::integral_constant<int, r>{}, asl[r]);
        };
        step(std::integral_constant<int, 0>{});
        step(std::integral_constant<int, 1>{});
    }
    wait_vmcnt<0>();

    // the FP64 16 x 16 result: lane holds rows 16 t + g + 4 i of column 16 u + l16 of output tile (t, u)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int cc = 16 * u + l16;
        if (cc >= 63) continue;
        const int jj = cc / 9, q = cc % 9;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * t + g + 4 * i;
                if (r >= ROWS) continue;
                const int a = r / 9, p = r % 9;
                const int cs = h[G + a * JT + jj];
                if (cs < 0) continue;
                double *cp = vC + (int64_t)cs * BB + p * B + q;
                *cp = beta == 0.0 ? alpha * acc[t][u][i] : scale_add(alpha, acc[t][u][i], beta, *cp);
            }
        }
    }
}

// ---------------------------------------------------------------- BF16 matrix-core tiles (b = 9)
// The same tiles (G = 4 or 8 rows x 7 columns of 9 x 9 blocks) computed on the
// matrix cores with v_mfma_f32_16x16x32_bf16.  Operands are pre-packed in BF16: every
// A block as 9 rows of 16 (the contraction index m = 0..8 then 7 zeros),
// every B block transposed the same way (row q holds B[m][q]), 288 bytes per
// block, so each MFMA operand of a lane is one aligned 16-byte LDS read.  Two
// consecutive entries form the K = 32 of one MFMA (16 per entry, 9 of them
// live).  The tile's 9 G output rows are ceil(9 G / 16) MFMA row tiles (48 rows for
// 36, 80 for 72: the rest padding), its 63 output columns 4 column tiles (64).  Absent A or B
// blocks are staged from a packed zero block.  Entries are copied into a
// per-wave LDS ring of four slots by one 16-byte LDS-DMA per block (18 lanes),
// one entry pair ahead of the multiply.  Products are exact in FP32 and summed
// in FP32 in the matrix core's order.
constexpr int kPackedBlock = 9 * 16;             // BF16 elements per packed block
constexpr int kPackedBytes = kPackedBlock * 2;   // 288

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// BUF: copies through buffer resources over the packed operands (a_bytes,
// b_bytes at most kBufMaxBytes); absent blocks read zeros past the resource.
template <int G, bool BUF = false>
__device__ inline void tile_mfma_bf16(int64_t tile, const int *__restrict__ hdr, const int64_t *__restrict__ ebeg,
                                      const int *__restrict__ ent, const unsigned short *__restrict__ pA,
                                      const unsigned short *__restrict__ pBt, const unsigned short *__restrict__ pz,
                                      double *__restrict__ vC, double alpha, double beta, lds_char_t *ring,
                                      unsigned a_bytes = 0, unsigned b_bytes = 0)
{
    constexpr int B = 9, JT = 7, BB = 81;
    constexpr int ROWS = 9 * G, RT = (ROWS + 15) / 16;   // output rows, MFMA row tiles
    constexpr int HS = G + G * JT, ES = G + JT, NB = G + JT;
    constexpr int SLOT = NB * kPackedBytes;          // bytes per ring slot (one entry)
    constexpr int NI = NB;                           // DMA loads per entry
    const int lane = threadIdx.x & 63, l16 = lane & 15, g = lane >> 4;
    const int e_of_lane = g >> 1, half = g & 1;      // which entry of the pair, which 16-byte half
    const int *h = hdr + tile * HS;

    const int64_t e0 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile] >> 32)) << 32);
    const int64_t e1 = __builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] & 0xffffffff)) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(ebeg[tile + 1] >> 32)) << 32);
    const int n = (int)(e1 - e0);                    // even
    const_as4<int> *entu = (const_as4<int> *)(ent + e0 * ES);

    // LDS byte offsets of this lane's operands inside a slot (-1: padding row / column)
    int aoff[RT], boff[4];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int r = 16 * t + l16;
        aoff[t] = r < ROWS ? (r / 9) * kPackedBytes + (r % 9) * 32 + half * 16 : -1;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int cc = 16 * u + l16;
        boff[u] = cc < 63 ? (G + cc / 9) * kPackedBytes + (cc % 9) * 32 + half * 16 : -1;
    }
    f32x4_t acc[RT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[t][u] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc((void *)pA, 0, (int)a_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc((void *)pBt, 0, (int)b_bytes, 0x00020000);
    // copy entry q into ring slot P (18 lanes x 16 bytes per block)
    auto issue = [&](auto P, int q) {
        lds_char_t *slot = ring + decltype(P)::value * SLOT;
        int sl[NB];
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) sl[blk] = entu[(int64_t)q * ES + blk];
        if constexpr (BUF) {
            // one lane mask for the entry; slot -1 gives offset 2^32 - 288, past the resource
            if (lane < kPackedBytes / 16) {
#pragma unroll
                for (int blk = 0; blk < NB; ++blk)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        blk < G ? rsA : rsB, (lds_void_t *)(slot + blk * kPackedBytes), 16,
                        (unsigned)sl[blk] * (unsigned)kPackedBytes + 16u * (unsigned)lane, 0, 0, 0);
            }
            return;
        }
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) {
            const unsigned short *src =
                sl[blk] >= 0 ? (blk < G ? pA : pBt) + (int64_t)sl[blk] * kPackedBlock : pz;
            if (lane < kPackedBytes / 16)
                __builtin_amdgcn_global_load_lds((const void *)(reinterpret_cast<const char *>(src) + 16 * lane),
                                                 (lds_void_t *)(slot + blk * kPackedBytes), 16, 0, 0);
        }
    };
    auto wait_for = [&](int later) {   // entries issued after the pair being waited for
        if (later >= 2) wait_vmcnt<2 * NI>();
        else wait_vmcnt<0>();
    };
    auto zero8 = []() {
        bf16x8_t z;
#pragma unroll
        for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
        return z;
    };
    // the pair of entries in slots (P, P + 1)
    auto compute = [&](auto P) {
        const lds_char_t *slot = ring + (decltype(P)::value + e_of_lane) * SLOT;
        bf16x8_t av[RT], bv[4];
#pragma unroll
        for (int t = 0; t < RT; ++t)
            av[t] = aoff[t] >= 0 ? *(const __attribute__((address_space(3))) bf16x8_t *)(slot + aoff[t]) : zero8();
#pragma unroll
        for (int u = 0; u < 4; ++u)
            bv[u] = boff[u] >= 0 ? *(const __attribute__((address_space(3))) bf16x8_t *)(slot + boff[u]) : zero8();
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[t], bv[u], acc[t][u], 0, 0, 0);
    };

    // ring of 4 slots: pair s in slots 2 (s % 2), 2 (s % 2) + 1; pair s + 1 loads meanwhile
    if (0 < n) {
        issue(std::integral_constant<int, 0>{}, 0);
        issue(std::integral_constant<int, 1>{}, 1);
    }
    for (int q0 = 0; q0 < n; q0 += 4) {
        auto step = [&](auto S) {   // S = 0: entries q0, q0 + 1 in slots 0, 1; S = 1: q0 + 2, q0 + 3 in 2, 3
            constexpr int s = decltype(S)::value;
            const int q = q0 + 2 * s;
            if (q >= n) return;
            const bool more = q + 2 < n;
            if (more) {
                issue(std::integral_constant<int, 2 * (1 - s)>{}, q + 2);
                issue(std::integral_constant<int, 2 * (1 - s) + 1>{}, q + 3);
            }
            wait_for(more ? 2 : 0);
            compute(std::integral_constant<int, 2 * s>{});
        };
        step(std::integral_constant<int, 0>{});
        step(std::integral_constant<int, 1>{});
    }

    // epilogue: lane holds rows 16 t + 4 g + i of column 16 u + l16 of tile (t, u)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int cc = 16 * u + l16;
        if (cc >= 63) continue;
        const int jj = cc / 9, q = cc % 9;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * t + 4 * g + i;
                if (r >= ROWS) continue;
                const int a = r / 9, p = r % 9;
                const int cs = h[G + a * JT + jj];
                if (cs < 0) continue;
                double *cp = vC + (int64_t)cs * BB + p * B + q;
                *cp = beta == 0.0 ? alpha * (double)acc[t][u][i] : scale_add(alpha, (double)acc[t][u][i], beta, *cp);
            }
        }
    }
}

}  // namespace bsm
