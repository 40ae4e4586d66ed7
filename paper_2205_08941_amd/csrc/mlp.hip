// Learned initial guess: pair descriptors, a three-layer perceptron with FP32
// training kernels and BF16 matrix-core inference, Adam, and block predictions.
//
// The network maps the 32-value descriptor of an atom pair to a b x b block
// correction of the Hotelling or LNV start (include/bsm_guess.h).  Its
// workload is small next to the block products (about 58 kFLOP per pair per
// forward pass), so the kernels aim at plain, deterministic data flow:
//   - training: one fused kernel runs forward and backward for tiles of 32
//     samples with all activations in LDS; every thread owns a fixed set of
//     parameter-gradient entries in registers, so no atomics are needed; each
//     workgroup writes its partial gradient once and a fixed-order reduction
//     adds the partials;
//   - inference (BF16): each wavefront pushes 16 samples through the three
//     layers with 16x16x16 BF16 MFMAs (FP32 accumulation), weights pre-packed
//     into the per-lane operand layout, activations staged in LDS.
#include "bsm_internal.h"
#include "bsm_guess.h"

#include <cmath>
#include <vector>

namespace bsm {
namespace {

constexpr int kD = BSM_DESC_DIM;    // descriptor length
constexpr int kH = BSM_MLP_WIDTH;   // hidden width
constexpr int kTS = 32;             // samples per training tile
constexpr int kNT = 256;            // threads per workgroup
constexpr int kMaxParts = 256;      // workgroups of a gradient launch

struct Offs {
    int64_t w1, b1, w2, b2, w3, b3, total;
};

__host__ __device__ inline Offs offsets(int M)
{
    Offs o;
    o.w1 = 0;
    o.b1 = (int64_t)kD * kH;
    o.w2 = o.b1 + kH;
    o.b2 = o.w2 + (int64_t)kH * kH;
    o.w3 = o.b2 + kH;
    o.b3 = o.w3 + (int64_t)kH * M;
    o.total = o.b3 + M;
    return o;
}

// Where a forward pass puts its outputs: Y[s][o], or FP64 blocks
// blocks[s][o] <- beta blocks[s][o] + scale y (beta == 0 overwrites).
struct Out {
    float *Y;
    double *blocks;
    double scale, beta;
};

__device__ inline void put(const Out &out, int64_t at, float y)
{
    if (out.Y) {
        out.Y[at] = y;
    } else {
        const double v = out.scale * (double)y;
        out.blocks[at] = out.beta == 0.0 ? v : out.beta * out.blocks[at] + v;
    }
}

// ------------------------------------------------------------------ descriptors

__device__ inline double dmul(double a, double b) { return __dmul_rn(a, b); }
__device__ inline double dadd(double a, double b) { return __dadd_rn(a, b); }

__device__ inline void min_image(const double *__restrict__ pos, double3 box, int i, int j, double r[3])
{
    const double bx[3] = {box.x, box.y, box.z};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double d = pos[3 * j + c] - pos[3 * i + c];
        r[c] = d - dmul(bx[c], rint(d / bx[c]));
    }
}

__device__ inline double norm2(const double r[3]) { return dadd(dadd(dmul(r[0], r[0]), dmul(r[1], r[1])), dmul(r[2], r[2])); }

// tetrahedral directions of the first diamond sublattice, before the 1 / sqrt 3
__constant__ double kTetra[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};

constexpr int kFrame = 24;   // doubles per atom frame
constexpr double kBond0 = 2.3512589712747505;   // 5.43 sqrt(3) / 4 rounded to FP64: the ideal Si-Si bond, Angstrom
// environment density of an ideal-lattice atom over a 6 A neighbour pattern: the five
// diamond shells inside 6 A (4, 12, 12, 6, 12 atoms at 5.43 sqrt(q) / 4 A, q = 3, 8, 11,
// 16, 19) weighted by exp(-d / 1.5 A)
constexpr double kRho0 = 2.751647885181917;

// Per atom (see the header): fr[24 i] = s, fr[24 i + 1 + 3 a + c] = e[a][c],
// fr[24 i + 13 + a] = l[a], fr[24 i + 17 + c] = c_i[c], fr[24 i + 20] = rho_i (the
// sum over the row's other atoms of exp(-d / 1.5 A), in column order).
__global__ void k_atom_frames(int n, const double *__restrict__ pos, double3 box, const int *__restrict__ rowptr,
                              const int *__restrict__ cols, double *__restrict__ fr, int *__restrict__ bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double bd[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    int bj[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
    double bv[4][3] = {};
    int found = 0;
    double rho = 0.0;
    for (int s = rowptr[i]; s < rowptr[i + 1]; ++s) {
        const int j = cols[s];
        if (j == i) continue;
        ++found;
        double r[3];
        min_image(pos, box, i, j, r);
        const double d2 = norm2(r);
        rho = dadd(rho, exp(-sqrt(d2) / 1.5));
        // insert (d2, j) into the sorted best-four list
        int at = 4;
        while (at > 0 && (d2 < bd[at - 1] || (d2 == bd[at - 1] && j < bj[at - 1]))) --at;
        if (at == 4) continue;
        for (int q = 3; q > at; --q) {
            bd[q] = bd[q - 1];
            bj[q] = bj[q - 1];
            for (int c = 0; c < 3; ++c) bv[q][c] = bv[q - 1][c];
        }
        bd[at] = d2;
        bj[at] = j;
        for (int c = 0; c < 3; ++c) bv[at][c] = r[c];
    }
    if (found < 4) {
        *bad = 1;
        return;
    }
    const double inv3 = 1.0 / sqrt(3.0);
    double u[4][3], dots[4][4];
    for (int q = 0; q < 4; ++q) {
        const double d = sqrt(bd[q]);
        for (int c = 0; c < 3; ++c) u[q][c] = bv[q][c] / d;
        for (int a = 0; a < 4; ++a)
            dots[q][a] = dadd(dadd(dmul(u[q][0], kTetra[a][0] * inv3), dmul(u[q][1], kTetra[a][1] * inv3)),
                              dmul(u[q][2], kTetra[a][2] * inv3));
    }
    double sA = 0.0, sB = 0.0;
    for (int q = 0; q < 4; ++q) {
        double mA = -INFINITY, mB = -INFINITY;
        for (int a = 0; a < 4; ++a) {
            mA = fmax(mA, dots[q][a]);
            mB = fmax(mB, -dots[q][a]);
        }
        sA = dadd(sA, mA);
        sB = dadd(sB, mB);
    }
    const double sg = sA >= sB ? 1.0 : -1.0;
    double *f = fr + kFrame * (int64_t)i;
    f[0] = sg;
    for (int a = 0; a < 4; ++a) {
        int best = 0;
        for (int q = 1; q < 4; ++q)
            if (sg * dots[q][a] > sg * dots[best][a]) best = q;
        for (int c = 0; c < 3; ++c) f[1 + 3 * a + c] = u[best][c];
        f[13 + a] = sqrt(bd[best]);
    }
    for (int c = 0; c < 3; ++c) f[17 + c] = dadd(dadd(dadd(bv[0][c], bv[1][c]), bv[2][c]), bv[3][c]) / 4.0;
    f[20] = rho;
}

__global__ void k_pair_desc(int64_t nnz, const int *__restrict__ rowidx, const int *__restrict__ cols,
                            const double *__restrict__ pos, double3 box, double rc, const double *__restrict__ fr,
                            float *__restrict__ X)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nnz) return;
    const int i = rowidx[s], j = cols[s];
    double r[3];
    min_image(pos, box, i, j, r);
    const double d = sqrt(norm2(r));
    double rh[3];
    for (int c = 0; c < 3; ++c) rh[c] = d > 0.0 ? r[c] / d : 0.0;
    const double *fi = fr + kFrame * (int64_t)i, *fj = fr + kFrame * (int64_t)j;
    float v[kD];
    for (int c = 0; c < 3; ++c) v[c] = (float)(r[c] / rc);
    v[3] = (float)(d / rc);
    v[4] = (float)(dmul(d / rc, d / rc));
    v[5] = (float)exp(-d / 1.5);
    v[6] = (float)fi[0];
    v[7] = (float)fj[0];
    for (int a = 0; a < 4; ++a) {
        v[8 + a] = (float)dadd(dadd(dmul(rh[0], fi[1 + 3 * a]), dmul(rh[1], fi[2 + 3 * a])), dmul(rh[2], fi[3 + 3 * a]));
        v[12 + a] = (float)dadd(dadd(dmul(rh[0], fj[1 + 3 * a]), dmul(rh[1], fj[2 + 3 * a])), dmul(rh[2], fj[3 + 3 * a]));
        v[16 + a] = (float)(10.0 * (fi[13 + a] - kBond0));
        v[20 + a] = (float)(10.0 * (fj[13 + a] - kBond0));
    }
    for (int c = 0; c < 3; ++c) {
        v[24 + c] = (float)(10.0 * fi[17 + c]);
        v[27 + c] = (float)(10.0 * fj[17 + c]);
    }
    v[30] = (float)(10.0 * (fi[20] - kRho0));
    v[31] = (float)(10.0 * (fj[20] - kRho0));
    float4 *o = reinterpret_cast<float4 *>(X + (int64_t)kD * s);
    for (int q = 0; q < kD / 4; ++q) o[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// ------------------------------------------------------------------ FP32 network

__device__ inline double wave_sum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Forward (GRAD = false: outputs to `out`) or forward + backward (GRAD = true:
// per-workgroup partial gradients and partial sums of squared residuals) over
// samples 0..n-1; sample s is row idx[s] of X and T (row s when idx is NULL).
// Thread t serves hidden / output unit o = t % 128 for samples of its half
// (t / 128) of the tile, and owns the gradient entries (k, o) with
// k = t / 128 + 2 r of every weight matrix: it alone reads and writes them in
// its workgroup's partial-gradient row, so the row needs no atomics.
template <bool GRAD>
__global__ __launch_bounds__(kNT) void k_mlp_f32(const float *__restrict__ prm, int M, int64_t n,
                                                 const float *__restrict__ X, const int *__restrict__ idx,
                                                 const float *__restrict__ T, float inv_n, Out out,
                                                 float *__restrict__ gpart, double *__restrict__ lpart)
{
    __shared__ float xs[kTS][kD];
    __shared__ float a1[kTS][kH];
    __shared__ float a2[kTS][kH];   // h2; in the backward pass dz1
    __shared__ float dy[kTS][kH];
    __shared__ float dz[kTS][kH];   // dz2
    __shared__ double lsum[kNT / 64];
    const Offs of = offsets(M);
    const float *W1 = prm + of.w1, *B1 = prm + of.b1, *W2 = prm + of.w2, *B2 = prm + of.b2, *W3 = prm + of.w3,
                *B3 = prm + of.b3;
    const int t = threadIdx.x, o = t & (kH - 1), half = t >> 7, sb = half * (kTS / 2);
    float *g = GRAD ? gpart + (int64_t)blockIdx.x * of.total : nullptr;
    bool first = true;   // the first tile of this workgroup stores, later tiles add
    auto acc_to = [&](int64_t at, float v) { g[at] = first ? v : g[at] + v; };
    double lacc = 0.0;
    const int64_t ntiles = (n + kTS - 1) / kTS;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t s0 = tile * kTS;
        const int cnt = (int)min((int64_t)kTS, n - s0);
        for (int e = t; e < kTS * kD; e += kNT) {
            const int s = e / kD, k = e % kD;
            float v = 0.f;
            if (s < cnt) {
                const int64_t src = idx ? (int64_t)idx[s0 + s] : s0 + s;
                v = X[src * kD + k];
            }
            xs[s][k] = v;
        }
        __syncthreads();
        float acc[16];
        {
            const float bb = B1[o];
#pragma unroll
            for (int s = 0; s < 16; ++s) acc[s] = bb;
#pragma unroll 4
            for (int k = 0; k < kD; ++k) {
                const float w = W1[k * kH + o];
#pragma unroll
                for (int s = 0; s < 16; ++s) acc[s] = fmaf(xs[sb + s][k], w, acc[s]);
            }
#pragma unroll
            for (int s = 0; s < 16; ++s) a1[sb + s][o] = tanhf(acc[s]);
        }
        __syncthreads();
        {
            const float bb = B2[o];
#pragma unroll
            for (int s = 0; s < 16; ++s) acc[s] = bb;
#pragma unroll 4
            for (int k = 0; k < kH; ++k) {
                const float w = W2[k * kH + o];
#pragma unroll
                for (int s = 0; s < 16; ++s) acc[s] = fmaf(a1[sb + s][k], w, acc[s]);
            }
#pragma unroll
            for (int s = 0; s < 16; ++s) a2[sb + s][o] = tanhf(acc[s]);
        }
        __syncthreads();
        if (o < M) {
            const float bb = B3[o];
#pragma unroll
            for (int s = 0; s < 16; ++s) acc[s] = bb;
#pragma unroll 4
            for (int k = 0; k < kH; ++k) {
                const float w = W3[k * M + o];
#pragma unroll
                for (int s = 0; s < 16; ++s) acc[s] = fmaf(a2[sb + s][k], w, acc[s]);
            }
        }
        if (!GRAD) {
            if (o < M)
                for (int s = 0; s < 16; ++s)
                    if (sb + s < cnt) put(out, (s0 + sb + s) * M + o, acc[s]);
            continue;   // the next tile's first barrier orders the LDS reuse
        }
        // ---- backward: dy = (y - t) / n
        if (o < M) {
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                float r = 0.f;
                if (sb + s < cnt) {
                    const int64_t src = idx ? (int64_t)idx[s0 + sb + s] : s0 + sb + s;
                    r = acc[s] - T[src * M + o];
                }
                lacc += (double)(r * r);
                dy[sb + s][o] = r * inv_n;
            }
        }
        __syncthreads();
        // dz2 = (dy W3^T) (1 - h2^2) for hidden unit o
#pragma unroll
        for (int s = 0; s < 16; ++s) acc[s] = 0.f;
#pragma unroll 4
        for (int m = 0; m < M; ++m) {
            const float w = W3[o * M + m];
#pragma unroll
            for (int s = 0; s < 16; ++s) acc[s] = fmaf(dy[sb + s][m], w, acc[s]);
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const float h = a2[sb + s][o];
            dz[sb + s][o] = acc[s] * (1.f - h * h);
        }
        if (o < M) {   // dW3 = h2^T dy, db3 = sum dy
            float col[kTS];
#pragma unroll
            for (int s = 0; s < kTS; ++s) col[s] = dy[s][o];
            for (int r = 0; r < 64; ++r) {
                const int k = half + 2 * r;
                float sum = 0.f;
#pragma unroll
                for (int s = 0; s < kTS; ++s) sum = fmaf(a2[s][k], col[s], sum);
                acc_to(of.w3 + (int64_t)k * M + o, sum);
            }
            if (half == 0) {
                float sum = 0.f;
                for (int s = 0; s < kTS; ++s) sum += col[s];
                acc_to(of.b3 + o, sum);
            }
        }
        __syncthreads();
        {   // dW2 = h1^T dz2, db2 = sum dz2
            float col[kTS];
#pragma unroll
            for (int s = 0; s < kTS; ++s) col[s] = dz[s][o];
            for (int r = 0; r < 64; ++r) {
                const int k = half + 2 * r;
                float sum = 0.f;
#pragma unroll
                for (int s = 0; s < kTS; ++s) sum = fmaf(a1[s][k], col[s], sum);
                acc_to(of.w2 + (int64_t)k * kH + o, sum);
            }
            if (half == 0) {
                float sum = 0.f;
                for (int s = 0; s < kTS; ++s) sum += col[s];
                acc_to(of.b2 + o, sum);
            }
        }
        // dz1 = (dz2 W2^T) (1 - h1^2) into a2 (h2 is no longer read)
#pragma unroll
        for (int s = 0; s < 16; ++s) acc[s] = 0.f;
#pragma unroll 4
        for (int m = 0; m < kH; ++m) {
            const float w = W2[o * kH + m];
#pragma unroll
            for (int s = 0; s < 16; ++s) acc[s] = fmaf(dz[sb + s][m], w, acc[s]);
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const float h = a1[sb + s][o];
            a2[sb + s][o] = acc[s] * (1.f - h * h);
        }
        __syncthreads();
        {   // dW1 = x^T dz1, db1 = sum dz1
            float col[kTS];
#pragma unroll
            for (int s = 0; s < kTS; ++s) col[s] = a2[s][o];
            for (int r = 0; r < kD / 2; ++r) {
                const int k = half + 2 * r;
                float sum = 0.f;
#pragma unroll
                for (int s = 0; s < kTS; ++s) sum = fmaf(xs[s][k], col[s], sum);
                acc_to(of.w1 + (int64_t)k * kH + o, sum);
            }
            if (half == 0) {
                float sum = 0.f;
                for (int s = 0; s < kTS; ++s) sum += col[s];
                acc_to(of.b1 + o, sum);
            }
        }
        first = false;
        __syncthreads();
    }
    if (GRAD) {
        lacc = wave_sum(lacc);
        if ((t & 63) == 0) lsum[t >> 6] = lacc;
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int w = 0; w < kNT / 64; ++w) s += lsum[w];
            lpart[blockIdx.x] = s;
        }
    }
}

// grad[p] = sum over parts w (ascending) of gpart[w][p]
__global__ void k_sum_partials(int64_t P, int parts, const float *__restrict__ gpart, float *__restrict__ grad)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float s = 0.f;
    for (int w = 0; w < parts; ++w) s += gpart[(int64_t)w * P + p];
    grad[p] = s;
}

// acc[0] (+)= scale * sum of the parts, in part order
__global__ void k_sum_loss(int parts, const double *__restrict__ lpart, double scale, int accumulate,
                           double *__restrict__ acc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int w = 0; w < parts; ++w) s += lpart[w];
    acc[0] = (accumulate ? acc[0] : 0.0) + scale * s;
}

__global__ void k_adam(int64_t P, float *__restrict__ prm, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    prm[p] -= lr * (mp * c1) / (sqrtf(vp * c2) + eps);
}

// ------------------------------------------------------------------ BF16 inference

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest even; NaN stays NaN, infinities stay infinite
__device__ inline unsigned short bf16_bits(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u | ((u & 0x007fffffu) ? 0x00400000u : 0u)) >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// Pack a K x N input-major weight matrix into the B-operand layout of the
// 16x16x16 BF16 MFMA: tile (kt, nt), lane l, element e holds
// W[16 kt + 4 (l / 16) + e][16 nt + l % 16] (zero outside the matrix).
__global__ void k_pack_bf16(const float *__restrict__ W, int K, int N, int KT, int NTl, unsigned short *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)KT * NTl * 256) return;
    const int e = (int)(q & 3), l = (int)((q >> 2) & 63);
    const int nt = (int)((q >> 8) % NTl), kt = (int)((q >> 8) / NTl);
    const int k = 16 * kt + 4 * (l >> 4) + e, c = 16 * nt + (l & 15);
    out[q] = (k < K && c < N) ? bf16_bits(W[(int64_t)k * N + c]) : (unsigned short)0;
}

constexpr int kHP = kH + 8;   // padded LDS row (bf16 elements)
constexpr int kKT1 = kD / 16;  // k-steps of the first layer

// 4 wavefronts x 16 samples.  For the 16x16x16 MFMA, lane l supplies row
// l % 16 of A (k = 4 (l / 16) .. + 3) and column l % 16 of B, and receives
// rows 4 (l / 16) .. + 3 of column l % 16 of the result.
__global__ __launch_bounds__(256) void k_mlp_bf16(const unsigned short *__restrict__ P1,
                                                  const unsigned short *__restrict__ P2,
                                                  const unsigned short *__restrict__ P3,
                                                  const float *__restrict__ B1, const float *__restrict__ B2,
                                                  const float *__restrict__ B3, int M, int NT3, int64_t n,
                                                  const float *__restrict__ X, Out out)
{
    __shared__ __align__(16) unsigned short h[4][16][kHP];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, m = l & 15, kq = l >> 4;
    const int64_t base = ((int64_t)blockIdx.x * 4 + w) * 16;
    unsigned short (*hw)[kHP] = h[w];
    const bf16x4 *p1 = reinterpret_cast<const bf16x4 *>(P1);
    const bf16x4 *p2 = reinterpret_cast<const bf16x4 *>(P2);
    const bf16x4 *p3 = reinterpret_cast<const bf16x4 *>(P3);
    // layer 1: K = kD (kKT1 steps of 16)
    f32x4 acc[8];
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < kKT1; ++kt) {
        bf16x4 a;
        const int64_t s = base + m;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (s < n) x = *reinterpret_cast<const float4 *>(X + s * kD + kt * 16 + 4 * kq);
        a[0] = (short)bf16_bits(x.x);
        a[1] = (short)bf16_bits(x.y);
        a[2] = (short)bf16_bits(x.z);
        a[3] = (short)bf16_bits(x.w);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, p1[(kt * 8 + nt) * 64 + l], acc[nt], 0, 0, 0);
    }
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
        const float bb = B1[nt * 16 + m];
#pragma unroll
        for (int e = 0; e < 4; ++e) hw[4 * kq + e][nt * 16 + m] = bf16_bits(tanhf(acc[nt][e] + bb));
    }
    __syncthreads();
    // layer 2: K = 128
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 8; ++kt) {
        const bf16x4 av = *reinterpret_cast<const bf16x4 *>(&hw[m][kt * 16 + 4 * kq]);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, p2[(kt * 8 + nt) * 64 + l], acc[nt], 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
        const float bb = B2[nt * 16 + m];
#pragma unroll
        for (int e = 0; e < 4; ++e) hw[4 * kq + e][nt * 16 + m] = bf16_bits(tanhf(acc[nt][e] + bb));
    }
    __syncthreads();
    // layer 3: K = 128, N = M (NT3 tiles of 16)
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 8; ++kt) {
        const bf16x4 av = *reinterpret_cast<const bf16x4 *>(&hw[m][kt * 16 + 4 * kq]);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
            if (nt < NT3)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, p3[(kt * NT3 + nt) * 64 + l], acc[nt], 0, 0, 0);
    }
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
        const int col = nt * 16 + m;
        if (nt >= NT3 || col >= M) continue;
        const float bb = B3[col];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t s = base + 4 * kq + e;
            if (s < n) put(out, s * M + col, acc[nt][e] + bb);
        }
    }
}

__global__ void k_fill_f64(int64_t n, double v, double *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_targets(int64_t n, const double *__restrict__ A, const double *__restrict__ B, double scale,
                          float *__restrict__ T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) T[i] = (float)((A[i] - B[i]) / scale);
}

unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace
}  // namespace bsm

using namespace bsm;

struct bsm_mlp_s {
    Context *c = nullptr;
    int M = 0;
    int64_t P = 0;
    DevBuf prm, m, v, grad, gpart, lpart, loss, pk1, pk2, pk3;
    bool packed = false;
    int64_t t = 0;   // Adam steps taken

    int nt3() const { return (M + 15) / 16; }

    void pack()
    {
        if (packed) return;
        const Offs of = offsets(M);
        hipStream_t st = c->stream;
        const float *p = prm.as<float>();
        k_pack_bf16<<<grid_for(kKT1 * 8 * 256, 256), 256, 0, st>>>(p + of.w1, kD, kH, kKT1, 8, pk1.as<unsigned short>());
        k_pack_bf16<<<grid_for(8 * 8 * 256, 256), 256, 0, st>>>(p + of.w2, kH, kH, 8, 8, pk2.as<unsigned short>());
        k_pack_bf16<<<grid_for((int64_t)8 * nt3() * 256, 256), 256, 0, st>>>(p + of.w3, kH, M, 8, nt3(),
                                                                            pk3.as<unsigned short>());
        BSM_HIP_TRY(hipGetLastError());
        packed = true;
    }

    void forward(int precision, int64_t n, const float *X, const Out &out)
    {
        BSM_REQUIRE(precision == BSM_F32 || precision == BSM_BF16, BSM_EINVAL, "precision must be BSM_F32 or BSM_BF16");
        if (n == 0) return;
        BSM_REQUIRE(reinterpret_cast<uintptr_t>(X) % 16 == 0, BSM_EINVAL, "X must be 16-byte aligned");
        hipStream_t st = c->stream;
        if (precision == BSM_F32) {
            const int64_t tiles = (n + kTS - 1) / kTS;
            const unsigned grid = (unsigned)std::min<int64_t>(tiles, 4096);
            k_mlp_f32<false><<<grid, kNT, 0, st>>>(prm.as<float>(), M, n, X, nullptr, nullptr, 0.f, out, nullptr,
                                                    nullptr);
        } else {
            pack();
            const Offs of = offsets(M);
            const float *p = prm.as<float>();
            k_mlp_bf16<<<grid_for(n, 64), 256, 0, st>>>(pk1.as<unsigned short>(), pk2.as<unsigned short>(),
                                                       pk3.as<unsigned short>(), p + of.b1, p + of.b2, p + of.b3, M,
                                                       nt3(), n, X, out);
        }
        BSM_HIP_TRY(hipGetLastError());
    }

    // gradient of the minibatch (n samples; rows idx[s] or s) into grad; the
    // loss sum (times `scale`) into loss[0], added when `accumulate`
    void loss_grad(int64_t n, const float *X, const int *idx, const float *T, double scale, int accumulate)
    {
        hipStream_t st = c->stream;
        const int64_t tiles = (n + kTS - 1) / kTS;
        const int parts = (int)std::min<int64_t>(tiles, kMaxParts);
        k_mlp_f32<true><<<parts, kNT, 0, st>>>(prm.as<float>(), M, n, X, idx, T, (float)(1.0 / (double)n),
                                                Out{nullptr, nullptr, 0.0, 0.0}, gpart.as<float>(),
                                                lpart.as<double>());
        k_sum_partials<<<grid_for(P, 256), 256, 0, st>>>(P, parts, gpart.as<float>(), grad.as<float>());
        k_sum_loss<<<1, 64, 0, st>>>(parts, lpart.as<double>(), scale, accumulate, loss.as<double>());
        BSM_HIP_TRY(hipGetLastError());
    }

    void adam(const bsm_adam &o, const float *g)
    {
        BSM_REQUIRE(o.lr > 0.f && o.beta1 >= 0.f && o.beta1 < 1.f && o.beta2 >= 0.f && o.beta2 < 1.f && o.eps >= 0.f,
                    BSM_EINVAL, "bad Adam parameters");
        ++t;
        const double c1 = 1.0 / (1.0 - std::pow((double)o.beta1, (double)t));
        const double c2 = 1.0 / (1.0 - std::pow((double)o.beta2, (double)t));
        k_adam<<<grid_for(P, 256), 256, 0, c->stream>>>(P, prm.as<float>(), m.as<float>(), v.as<float>(), g, o.lr,
                                                        o.beta1, o.beta2, o.eps, (float)c1, (float)c2);
        BSM_HIP_TRY(hipGetLastError());
        packed = false;
    }

    void clear_adam()
    {
        hipStream_t st = c->stream;
        BSM_HIP_TRY(hipMemsetAsync(m.ptr, 0, sizeof(float) * P, st));
        BSM_HIP_TRY(hipMemsetAsync(v.ptr, 0, sizeof(float) * P, st));
        t = 0;
    }
};

#define MLP_TRY try {
#define MLP_CATCH                                                  \
    }                                                              \
    catch (const Error &e) { return fail(e.code, e.msg); }         \
    catch (...) { return fail(BSM_EINVAL, "unknown error"); }

extern "C" {

int64_t bsm_mlp_param_count(const bsm_mlp_shape *shape)
{
    if (!shape || shape->width != kH || shape->out_dim < 1 || shape->out_dim > kH) return BSM_EINVAL;
    return offsets(shape->out_dim).total;
}

int bsm_mlp_create(bsm_ctx ctx, const bsm_mlp_shape *shape, const float *params, bsm_mlp *out)
{
    MLP_TRY
    BSM_REQUIRE(ctx && shape && params && out, BSM_EINVAL, "NULL argument");
    BSM_REQUIRE(shape->width == kH, BSM_EINVAL, "hidden width must be 128");
    BSM_REQUIRE(shape->out_dim >= 1 && shape->out_dim <= kH, BSM_EINVAL, "out_dim must be 1..128");
    std::unique_ptr<bsm_mlp_s> net(new bsm_mlp_s());
    Context *c = &ctx->c;
    net->c = c;
    net->M = shape->out_dim;
    net->P = offsets(net->M).total;
    const size_t pb = sizeof(float) * (size_t)net->P;
    net->prm = DevBuf(c, pb);
    net->m = DevBuf(c, pb);
    net->v = DevBuf(c, pb);
    net->grad = DevBuf(c, pb);
    net->gpart = DevBuf(c, pb * kMaxParts);
    net->lpart = DevBuf(c, sizeof(double) * kMaxParts);
    net->loss = DevBuf(c, sizeof(double) * 2);
    net->pk1 = DevBuf(c, sizeof(unsigned short) * kKT1 * 8 * 256);
    net->pk2 = DevBuf(c, sizeof(unsigned short) * 8 * 8 * 256);
    net->pk3 = DevBuf(c, sizeof(unsigned short) * 8 * (size_t)net->nt3() * 256);
    BSM_HIP_TRY(hipMemcpyAsync(net->prm.ptr, params, pb, hipMemcpyHostToDevice, c->stream));
    net->clear_adam();
    BSM_HIP_TRY(hipStreamSynchronize(c->stream));
    *out = net.release();
    return BSM_OK;
    MLP_CATCH
}

int bsm_mlp_get_params(bsm_mlp net, float *params)
{
    MLP_TRY
    BSM_REQUIRE(net && params, BSM_EINVAL, "NULL argument");
    BSM_HIP_TRY(hipMemcpyAsync(params, net->prm.ptr, sizeof(float) * net->P, hipMemcpyDeviceToHost, net->c->stream));
    BSM_HIP_TRY(hipStreamSynchronize(net->c->stream));
    return BSM_OK;
    MLP_CATCH
}

int bsm_mlp_set_params(bsm_mlp net, const float *params)
{
    MLP_TRY
    BSM_REQUIRE(net && params, BSM_EINVAL, "NULL argument");
    BSM_HIP_TRY(hipMemcpyAsync(net->prm.ptr, params, sizeof(float) * net->P, hipMemcpyHostToDevice, net->c->stream));
    net->clear_adam();
    net->packed = false;
    BSM_HIP_TRY(hipStreamSynchronize(net->c->stream));
    return BSM_OK;
    MLP_CATCH
}

int bsm_mlp_destroy(bsm_mlp net)
{
    if (net) {
        (void)hipStreamSynchronize(net->c->stream);
        delete net;
    }
    return BSM_OK;
}

int bsm_pair_descriptors(bsm_ctx ctx, bsm_pattern NP, bsm_pattern P, float *desc)
{
    MLP_TRY
    BSM_REQUIRE(ctx && NP && P && desc, BSM_EINVAL, "NULL argument");
    BSM_REQUIRE(reinterpret_cast<uintptr_t>(desc) % 16 == 0, BSM_EINVAL, "desc must be 16-byte aligned");
    BSM_REQUIRE(NP->natoms == P->natoms && NP->box[0] == P->box[0] && NP->box[1] == P->box[1] &&
                    NP->box[2] == P->box[2],
                BSM_EPATTERN, "neighbour pattern is over other atoms");
    Context *c = &ctx->c;
    hipStream_t st = c->stream;
    const int n = P->natoms;
    const double3 box = make_double3(P->box[0], P->box[1], P->box[2]);
    DevBuf fr(c, sizeof(double) * kFrame * (size_t)std::max(1, n)), bad(c, sizeof(int));
    BSM_HIP_TRY(hipMemsetAsync(bad.ptr, 0, sizeof(int), st));
    k_atom_frames<<<grid_for(n, 128), 128, 0, st>>>(n, NP->pos.as<double>(), box, NP->rowptr.as<int>(),
                                                    NP->cols.as<int>(), fr.as<double>(), bad.as<int>());
    BSM_HIP_TRY(hipGetLastError());
    int hbad = 0;
    BSM_HIP_TRY(hipMemcpyAsync(&hbad, bad.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
    BSM_HIP_TRY(hipStreamSynchronize(st));
    BSM_REQUIRE(!hbad, BSM_EINVAL, "an atom has fewer than four neighbours in the neighbour pattern");
    if (P->nnzb > 0)
        k_pair_desc<<<grid_for(P->nnzb, 256), 256, 0, st>>>(P->nnzb, P->rowidx.as<int>(), P->cols.as<int>(),
                                                            P->pos.as<double>(), box, P->cutoff, fr.as<double>(),
                                                            desc);
    BSM_HIP_TRY(hipGetLastError());
    BSM_HIP_TRY(hipStreamSynchronize(st));   // the frames buffer is released on return
    return BSM_OK;
    MLP_CATCH
}

int bsm_mlp_forward(bsm_mlp net, int precision, int64_t n, const float *X, float *Y)
{
    MLP_TRY
    BSM_REQUIRE(net && n >= 0 && (n == 0 || (X && Y)), BSM_EINVAL, "bad argument");
    net->forward(precision, n, X, Out{Y, nullptr, 0.0, 0.0});
    return BSM_OK;
    MLP_CATCH
}

int bsm_mlp_loss_grad(bsm_mlp net, int64_t n, const float *X, const float *T, double *loss, float *grad)
{
    MLP_TRY
    BSM_REQUIRE(net && X && T && grad && n >= 1, BSM_EINVAL, "bad argument");
    net->loss_grad(n, X, nullptr, T, 0.5 / (double)n, 0);
    BSM_HIP_TRY(hipMemcpyAsync(grad, net->grad.ptr, sizeof(float) * net->P, hipMemcpyDeviceToDevice, net->c->stream));
    double h = 0.0;
    BSM_HIP_TRY(hipMemcpyAsync(&h, net->loss.ptr, sizeof(double), hipMemcpyDeviceToHost, net->c->stream));
    BSM_HIP_TRY(hipStreamSynchronize(net->c->stream));
    if (loss) *loss = h;
    return BSM_OK;
    MLP_CATCH
}

int bsm_mlp_adam_step(bsm_mlp net, const bsm_adam *opt, const float *grad)
{
    MLP_TRY
    BSM_REQUIRE(net && opt && grad, BSM_EINVAL, "NULL argument");
    net->adam(*opt, grad);
    return BSM_OK;
    MLP_CATCH
}

int bsm_mlp_train(bsm_mlp net, const bsm_mlp_train_params *p, int64_t n, const float *X, const float *T,
                  const int32_t *perm, double *epoch_loss)
{
    MLP_TRY
    BSM_REQUIRE(net && p && X && T && n >= 1, BSM_EINVAL, "bad argument");
    BSM_REQUIRE(p->epochs >= 0 && p->batch >= 1, BSM_EINVAL, "bad epochs or batch");
    hipStream_t st = net->c->stream;
    const int64_t nb = (n + p->batch - 1) / p->batch;
    for (int e = 0; e < p->epochs; ++e) {
        for (int64_t k = 0; k < nb; ++k) {
            const int64_t s0 = k * p->batch, cnt = std::min<int64_t>(p->batch, n - s0);
            const double scale = 0.5 / (double)cnt / (double)nb;   // mean over minibatches
            if (perm)
                net->loss_grad(cnt, X, perm + s0, T, scale, k > 0);
            else
                net->loss_grad(cnt, X + s0 * kD, nullptr, T + s0 * net->M, scale, k > 0);
            net->adam(p->opt, net->grad.as<float>());
        }
        double h = 0.0;
        BSM_HIP_TRY(hipMemcpyAsync(&h, net->loss.ptr, sizeof(double), hipMemcpyDeviceToHost, st));
        BSM_HIP_TRY(hipStreamSynchronize(st));
        if (epoch_loss) epoch_loss[e] = h;
    }
    return BSM_OK;
    MLP_CATCH
}

int bsm_mlp_targets(bsm_ctx ctx, const bsm_matrix *A, const bsm_matrix *B, double scale, float *T)
{
    MLP_TRY
    BSM_REQUIRE(ctx && T, BSM_EINVAL, "NULL argument");
    check_matrix(A, "A");
    check_matrix(B, "B");
    BSM_REQUIRE(A->pattern == B->pattern, BSM_EPATTERN, "A and B must share a pattern");
    BSM_REQUIRE(scale != 0.0 && std::isfinite(scale), BSM_EINVAL, "scale must be finite and non-zero");
    const int64_t ne = nelems(A->pattern);
    if (ne > 0)
        k_targets<<<grid_for(ne, 256), 256, 0, ctx->c.stream>>>(ne, (const double *)A->blocks,
                                                              (const double *)B->blocks, scale, T);
    BSM_HIP_TRY(hipGetLastError());
    return BSM_OK;
    MLP_CATCH
}

int bsm_mlp_predict_blocks(bsm_mlp net, int precision, const float *X, double scale, double beta,
                           const bsm_matrix *M)
{
    MLP_TRY
    BSM_REQUIRE(net && X, BSM_EINVAL, "NULL argument");
    check_matrix(M, "M");
    const int b = M->pattern->b;
    BSM_REQUIRE(b * b == net->M, BSM_EPATTERN, "network out_dim must be b^2");
    net->forward(precision, M->pattern->nnzb, X, Out{nullptr, (double *)M->blocks, scale, beta});
    return BSM_OK;
    MLP_CATCH
}

}  // extern "C"
