/*
 * FP64 CPU oracle for the block-sparse linear-scaling hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct loops that define
 * what the HIP library must compute.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path never
 * does.  It shares no source with the HIP library.
 *
 * The paper (Background and Current Status) describes the solver as built on
 * "sparse matrix storage and operations" exploiting locality: matrices are
 * stored as atom blocks kept only for atom pairs closer than a cutoff.  The
 * operations below are the textbook definitions of those objects:
 *
 *   pattern P_r      = { (i, j) : minimum-image distance d_ij < r } plus i == j
 *   mask_C(A B)_ij   = sum over k with (i,k) in P_A and (k,j) in P_B of A_ik B_kj,
 *                      kept for (i, j) in P_C only
 *   Tr(A B)          = sum over (i,k) in P_A of sum_pq A_ik[p][q] B_ki[q][p]
 *
 * Storage: block CSR.  rowptr[n+1] (int64), cols[nnz] (int32, ascending within
 * a row), vals[nnz * b * b] (row-major b x b per block, in CSR order).
 *
 * Build: gcc -O3 -march=native -fopenmp -ffp-contract=off -shared -fPIC (no FMA contraction,
 * so distances are rounded exactly as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* squared minimum-image distance between atoms i and j of an orthorhombic box */
static double min_image_d2(const double *pos, const double *box, int i, int j)
{
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double d = pos[3 * j + c] - pos[3 * i + c];
        double s = nearbyint(d / box[c]);
        d = d - s * box[c];
        d2 = d2 + d * d;
    }
    return d2;
}

/* Pattern, first pass: number of columns of every row (brute force over all pairs). */
int64_t orc_pattern_count(int n, const double *pos, const double *box, double r,
                          int64_t *rowcount)
{
    int64_t total = 0;
    double r2 = r * r;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int j = 0; j < n; ++j)
            if (j == i || min_image_d2(pos, box, i, j) < r2)
                ++c;
        rowcount[i] = c;
        total += c;
    }
    return total;
}

/* Pattern, second pass: fill columns in ascending order; rowptr from the counts. */
void orc_pattern_fill(int n, const double *pos, const double *box, double r,
                      const int64_t *rowptr, int32_t *cols)
{
    double r2 = r * r;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        int64_t p = rowptr[i];
        for (int j = 0; j < n; ++j)
            if (j == i || min_image_d2(pos, box, i, j) < r2)
                cols[p++] = j;
    }
}

/* slot of (i, j) in a pattern, or -1: binary search in row i */
static int64_t find_slot(const int64_t *rowptr, const int32_t *cols, int i, int j)
{
    int64_t lo = rowptr[i], hi = rowptr[i + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cols[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < rowptr[i + 1] && cols[lo] == j) ? lo : -1;
}

int64_t orc_find_slot(const int64_t *rowptr, const int32_t *cols, int i, int j)
{
    return find_slot(rowptr, cols, i, j);
}

/*
 * C <- alpha * mask_C(A B) + beta * C for rows [row_begin, row_end).
 * beta == 0 overwrites C (old contents ignored).  Every block triple
 * (i,k,j) with (i,k) in A, (k,j) in B, (i,j) in C is visited once; the sum
 * over k runs in ascending k, then ascending j inside row k of B.
 */
void orc_multiply(int n, int b, double alpha,
                  const int64_t *rpA, const int32_t *cA, const double *vA,
                  const int64_t *rpB, const int32_t *cB, const double *vB,
                  double beta,
                  const int64_t *rpC, const int32_t *cC, double *vC,
                  int row_begin, int row_end)
{
    const int bb = b * b;
#pragma omp parallel
    {
        int64_t *where = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        int64_t maxrow = 0;
        for (int i = row_begin; i < row_end; ++i)
            if (rpC[i + 1] - rpC[i] > maxrow) maxrow = rpC[i + 1] - rpC[i];
        double *acc = (double *)malloc(sizeof(double) * (size_t)(maxrow > 0 ? maxrow : 1) * bb);
        for (int j = 0; j < n; ++j) where[j] = -1;
#pragma omp for schedule(dynamic, 1)
        for (int i = row_begin; i < row_end; ++i) {
            int64_t c0 = rpC[i], c1 = rpC[i + 1];
            for (int64_t s = c0; s < c1; ++s) where[cC[s]] = s - c0;
            memset(acc, 0, sizeof(double) * (size_t)(c1 - c0) * bb);
            for (int64_t sa = rpA[i]; sa < rpA[i + 1]; ++sa) {
                int k = cA[sa];
                const double *a = vA + sa * bb;
                for (int64_t sb = rpB[k]; sb < rpB[k + 1]; ++sb) {
                    int64_t t = where[cB[sb]];
                    if (t < 0) continue;
                    const double *bk = vB + sb * bb;
                    double *c = acc + t * bb;
                    /* c[p][q] += sum over m of a[p][m] bk[m][q], each sum
                       started at zero and taken in ascending m; the q sums of
                       one p are carried side by side */
                    for (int p = 0; p < b; ++p) {
                        double sum[b];
                        for (int q = 0; q < b; ++q) sum[q] = 0.0;
                        for (int m = 0; m < b; ++m) {
                            const double apm = a[p * b + m];
                            for (int q = 0; q < b; ++q) sum[q] += apm * bk[m * b + q];
                        }
                        for (int q = 0; q < b; ++q) c[p * b + q] += sum[q];
                    }
                }
            }
            for (int64_t s = c0; s < c1; ++s) {
                double *out = vC + s * bb;
                const double *src = acc + (s - c0) * bb;
                for (int e = 0; e < bb; ++e)
                    out[e] = (beta == 0.0) ? alpha * src[e] : alpha * src[e] + beta * out[e];
                where[cC[s]] = -1;
            }
        }
        free(acc);
        free(where);
    }
}

/*
 * Number of block triples (i,k,j) visited by mask_C(A B), per row of C.
 * The algorithmic flop count of the product is 2 b^3 times their sum.
 */
void orc_count_triples(int n, const int64_t *rpA, const int32_t *cA,
                       const int64_t *rpB, const int32_t *cB,
                       const int64_t *rpC, const int32_t *cC, int64_t *per_row)
{
#pragma omp parallel
    {
        char *in_c = (char *)calloc((size_t)n, 1);
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < n; ++i) {
            for (int64_t s = rpC[i]; s < rpC[i + 1]; ++s) in_c[cC[s]] = 1;
            int64_t cnt = 0;
            for (int64_t sa = rpA[i]; sa < rpA[i + 1]; ++sa) {
                int k = cA[sa];
                for (int64_t sb = rpB[k]; sb < rpB[k + 1]; ++sb) cnt += in_c[cB[sb]];
            }
            per_row[i] = cnt;
            for (int64_t s = rpC[i]; s < rpC[i + 1]; ++s) in_c[cC[s]] = 0;
        }
        free(in_c);
    }
}

/*
 * Tr(A B) = sum_i sum_{(i,k) in A} sum_{p,q} A_ik[p][q] * B_ki[q][p], blocks of B
 * missing from its pattern being zero.  Per-row partial sums are added in row
 * order, so the result does not depend on the thread count.
 */
double orc_trace_product(int n, int b,
                         const int64_t *rpA, const int32_t *cA, const double *vA,
                         const int64_t *rpB, const int32_t *cB, const double *vB)
{
    const int bb = b * b;
    double *part = (double *)calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t sa = rpA[i]; sa < rpA[i + 1]; ++sa) {
            int k = cA[sa];
            int64_t sb = find_slot(rpB, cB, k, i);
            if (sb < 0) continue;
            const double *a = vA + sa * bb, *bk = vB + sb * bb;
            for (int p = 0; p < b; ++p)
                for (int q = 0; q < b; ++q) s += a[p * b + q] * bk[q * b + p];
        }
        part[i] = s;
    }
    double total = 0.0;
    for (int i = 0; i < n; ++i) total += part[i];
    free(part);
    return total;
}

/* ---------------------------------------------------------------------------
 * Mixed precision: each input element rounded to FP32 or BF16 (round to
 * nearest, ties to even), products accumulated in FP32 with fused
 * multiply-adds over k ascending, then m ascending, per output element;
 * the FP32 sum is widened exactly to FP64 and C <- alpha sum + beta C in FP64.
 * prec: 1 = FP32, 2 = BF16.
 */
static float round_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {          /* Inf stays Inf; NaN stays a (quiet) NaN */
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
        u &= 0xffff0000u;
    }
    float y;
    memcpy(&y, &u, 4);
    return y;
}

float orc_round_bf16(float x) { return round_bf16(x); }

static float round_in(double x, int prec)
{
    float f = (float)x;
    return prec == 2 ? round_bf16(f) : f;
}

void orc_multiply_mixed(int n, int b, int prec, double alpha,
                        const int64_t *rpA, const int32_t *cA, const double *vA,
                        const int64_t *rpB, const int32_t *cB, const double *vB,
                        double beta,
                        const int64_t *rpC, const int32_t *cC, double *vC,
                        int row_begin, int row_end)
{
    const int bb = b * b;
#pragma omp parallel
    {
        int64_t *where = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        int64_t maxrow = 0;
        for (int i = row_begin; i < row_end; ++i)
            if (rpC[i + 1] - rpC[i] > maxrow) maxrow = rpC[i + 1] - rpC[i];
        float *acc = (float *)malloc(sizeof(float) * (size_t)(maxrow > 0 ? maxrow : 1) * bb);
        float a[256], bk[256];
        for (int j = 0; j < n; ++j) where[j] = -1;
#pragma omp for schedule(dynamic, 1)
        for (int i = row_begin; i < row_end; ++i) {
            int64_t c0 = rpC[i], c1 = rpC[i + 1];
            for (int64_t s = c0; s < c1; ++s) where[cC[s]] = s - c0;
            memset(acc, 0, sizeof(float) * (size_t)(c1 - c0) * bb);
            for (int64_t sa = rpA[i]; sa < rpA[i + 1]; ++sa) {
                int k = cA[sa];
                for (int e = 0; e < bb; ++e) a[e] = round_in(vA[sa * bb + e], prec);
                for (int64_t sb = rpB[k]; sb < rpB[k + 1]; ++sb) {
                    int64_t t = where[cB[sb]];
                    if (t < 0) continue;
                    for (int e = 0; e < bb; ++e) bk[e] = round_in(vB[sb * bb + e], prec);
                    float *c = acc + t * bb;
                    for (int p = 0; p < b; ++p)
                        for (int q = 0; q < b; ++q)
                            for (int m = 0; m < b; ++m) c[p * b + q] = fmaf(a[p * b + m], bk[m * b + q], c[p * b + q]);
                }
            }
            for (int64_t s = c0; s < c1; ++s) {
                double *out = vC + s * bb;
                const float *src = acc + (s - c0) * bb;
                for (int e = 0; e < bb; ++e)
                    out[e] = (beta == 0.0) ? alpha * (double)src[e] : alpha * (double)src[e] + beta * out[e];
                where[cC[s]] = -1;
            }
        }
        free(acc);
        free(where);
    }
}
