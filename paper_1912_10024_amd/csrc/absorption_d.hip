// Coefficients of the absorption branch of Eq. 3 (the frequency -w of its
// integral over signed frequencies) from the combined coefficient table of the
// opposite component: for real displacement fields D<_ab(q, -w) = D>_ba(-q, w),
// and the bracket D_ba - D_bb - D_aa + D_ab is symmetric in a <-> b, so
//   Dm[q, w, a, n, i, j] = Dopp[(-q) mod Nqz, w, a, n, j, i].
// A permutation of complex entries: bit for bit, one thread per output entry.
#include <algorithm>

#include "sse_kernels.h"

namespace sse {

__global__ void absorption_d_kernel(Dims d, const double* __restrict__ Dopp, double* __restrict__ Dm) {
    const int64_t per_q = d.nw * d.na * d.nb * 9;  // complex entries per momentum
    const int64_t total = d.nqz * per_q;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = x / per_q, rest = x % per_q;
        const int ij = (int)(rest % 9);
        const int64_t qs = (d.nqz - q) % d.nqz;
        cstore(Dm, x, cload(Dopp, qs * per_q + (rest - ij) + (ij % 3) * 3 + ij / 3));
    }
}

hipError_t launch_absorption_d(const Dims& d, const double* Dopp, double* Dm, hipStream_t stream) {
    const int64_t total = d.nqz * d.nw * d.na * d.nb * 9;
    const unsigned groups = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(absorption_d_kernel, dim3(groups), dim3(256), 0, stream, d, Dopp, Dm);
    return hipGetLastError();
}

}  // namespace sse
