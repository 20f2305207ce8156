// Calibration library (libtgo_probe.so), separate from the product library:
// an integer issue probe whose counter run gives the number of 32-bit VALU
// instructions a CU of the device issues per clock, the peak the ALU-bound
// roofline of the enumeration kernels is priced against.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tgo_probe.h"

// eight independent shift-and-add chains per lane, no memory traffic
__global__ __launch_bounds__(256) void tgo_valu_probe_kernel(uint32_t *out, int iters, uint32_t s) {
    uint32_t a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = threadIdx.x ^ (uint32_t)j;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (a[j] >> 1) + s;
        s = s * 3u + 1u;
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r += a[j];
    if (r == 0x9e3779b9u) out[0] = r;  // practically never: keeps the chains live
}

extern "C" int tgo_probe_valu(int blocks, int iters, void *d_sink, void *stream) {
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20) || !d_sink) return -1;
    hipLaunchKernelGGL(tgo_valu_probe_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (uint32_t *)d_sink,
                       iters, 7u);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}
