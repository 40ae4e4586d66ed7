#include <hip/hip_runtime.h>
#include <utility>
template <int IDX>
__device__ inline double bcast(const double (&av)[6]) {
    return __builtin_amdgcn_mov_dpp(av[IDX / 16], 0x150 + (IDX % 16), 0xf, 0xf, true);
}
template <int R, int... M>
__device__ inline void row(double &acc, const double (&av)[6], const double (&bv)[9], std::integer_sequence<int, M...>) {
    ((acc = __builtin_fma(bcast<R * 9 + M>(av), bv[M], acc)), ...);
}
template <int... R>
__device__ inline void all(double (&acc)[9], const double (&av)[6], const double (&bv)[9], std::integer_sequence<int, R...>) {
    (row<R>(acc[R], av, bv, std::make_integer_sequence<int, 9>{}), ...);
}
__global__ void k(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c) {
    int l = threadIdx.x;
    double av[6]; for (int v = 0; v < 6; ++v) av[v] = a[(l & 15) + 16 * v];
    double bv[9]; for (int m = 0; m < 9; ++m) bv[m] = b[l * 9 + m];
    double acc[9] = {0};
    all(acc, av, bv, std::make_integer_sequence<int, 9>{});
    for (int r = 0; r < 9; ++r) c[l * 9 + r] = acc[r];
}
