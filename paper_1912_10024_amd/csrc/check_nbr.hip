// Range check of the neighbour table (every entry must index an atom).
#include "sse_kernels.h"

namespace sse {

__global__ void check_nbr_kernel(int64_t count, int64_t na, const int32_t* __restrict__ nbr, int* flag) {
    int bad = 0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < count; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = nbr[x];
        bad |= (v < 0 || v >= na);
    }
    if (__any(bad) && (threadIdx.x % 64) == 0) atomicOr(flag, 1);
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

hipError_t launch_check_nbr(const Dims& d, const int32_t* nbr, int* flag, hipStream_t stream) {
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, stream, flag);
    const int64_t count = d.na * d.nb;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(check_nbr_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, count, d.na, nbr, flag);
    return hipGetLastError();
}

}  // namespace sse
