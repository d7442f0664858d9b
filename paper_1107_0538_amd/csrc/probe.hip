// Bandwidth probe: the STREAM triad c = a + s b in FP64, used to measure the
// HBM bandwidth that a plain streaming kernel reaches on this device, against
// which the solver's kernels are also reported (besides the 8 TB/s peak).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/jpcg_probe.h"

namespace {

// Two FP64 values per thread per step (16-byte loads and stores), grid-stride.
__global__ __launch_bounds__(256) void k_triad(const double2* __restrict__ a, const double2* __restrict__ b,
                                               double2* __restrict__ c, double s, int64_t n2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 x = a[i], y = b[i];
        c[i] = make_double2(__builtin_fma(s, y.x, x.x), __builtin_fma(s, y.y, x.y));
    }
}

__global__ void k_triad_tail(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c,
                             double s, int64_t i)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) c[i] = __builtin_fma(s, b[i], a[i]);
}

}  // namespace

extern "C" int jpcg_stream_triad(const double* a, const double* b, double* c, double s, int64_t n, int32_t grid,
                                 void* hip_stream)
{
    if (n < 0 || (n > 0 && (!a || !b || !c))) return -1;
    if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) return -1;
    if (n == 0) return 0;
    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t n2 = n / 2;
    if (grid <= 0) grid = 4096;
    if (n2 > 0)
        hipLaunchKernelGGL(k_triad, dim3(grid), dim3(256), 0, st, (const double2*)a, (const double2*)b, (double2*)c,
                           s, n2);
    if (n & 1) hipLaunchKernelGGL(k_triad_tail, dim3(1), dim3(64), 0, st, a, b, c, s, n - 1);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
