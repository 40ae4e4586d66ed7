#include <hip/hip_runtime.h>
__global__ void k(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c) {
    int l = threadIdx.x;
    double av = a[l & 15];
    double bv = b[l];
    double acc = 0.0;
    asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:3 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(av), "v"(bv));
    c[l] = acc;
}
