#include <hip/hip_runtime.h>
template <int L>
__device__ inline void fdpp(double &acc, double a, double b) {
    asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(a), "v"(b), "n"(L));
}
__global__ void k(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c) {
    int l = threadIdx.x;
    double av = a[l & 15];
    double bv = b[l];
    double acc = 0.0;
    asm volatile("s_nop 1");
    fdpp<3>(acc, av, bv);
    fdpp<15>(acc, av, bv);
    c[l] = acc;
}
