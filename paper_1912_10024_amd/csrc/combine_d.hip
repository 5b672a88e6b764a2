// The bracket of Eq. 3, D_ba - D_bb - D_aa + D_ab, formed per neighbour slot
// from the phonon Green's function blocks [nqz][nw][na][nb+1][3][3] (slot 0 =
// D_aa, slot 1+n = the block of a with its n-th neighbour).  D_ba is read from
// b's own row at the slot where a appears, so the neighbour table must be
// symmetric; the reverse slots are found first and checked on the host.
#include "sse_kernels.h"

namespace sse {

__global__ void reverse_slot_kernel(int64_t na, int64_t nb, const int32_t* __restrict__ nbr, int32_t* rslot, int* flag) {
    int bad = 0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < na * nb; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = x / nb;
        const int32_t b = nbr[x];
        int32_t m = -1;
        if (b >= 0 && b < na)
            for (int64_t t = 0; t < nb; ++t)
                if (nbr[b * nb + t] == a) {
                    m = (int32_t)t;
                    break;
                }
        rslot[x] = m;
        bad |= (m < 0);
    }
    if (__any(bad) && (threadIdx.x % 64) == 0) atomicOr(flag, 1);
}

__global__ void combine_d_kernel(Dims d, const double* __restrict__ Df, const int32_t* __restrict__ nbr,
                                 const int32_t* __restrict__ rslot, double* __restrict__ Dc) {
    const int64_t S = d.nb + 1;
    const int64_t total = d.nqz * d.nw * d.na * d.nb * 9;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ij = x % 9, n = (x / 9) % d.nb, a = (x / (9 * d.nb)) % d.na, qw = x / (9 * d.nb * d.na);
        const int64_t b = nbr[a * d.nb + n], m = rslot[a * d.nb + n];
        const int64_t base = qw * d.na;
        const cd Dba = cload(Df, ((base + b) * S + 1 + m) * 9 + ij);
        const cd Dbb = cload(Df, ((base + b) * S) * 9 + ij);
        const cd Daa = cload(Df, ((base + a) * S) * 9 + ij);
        const cd Dab = cload(Df, ((base + a) * S + 1 + n) * 9 + ij);
        cd v;
        v.re = ((Dba.re - Dbb.re) - Daa.re) + Dab.re;
        v.im = ((Dba.im - Dbb.im) - Daa.im) + Dab.im;
        cstore(Dc, x, v);
    }
}

__global__ void zero_flag_kernel(int* p) { *p = 0; }

size_t combine_workspace_bytes(const Dims& d) { return 256 + sizeof(int32_t) * (size_t)(d.na * d.nb); }

hipError_t launch_reverse_slots(const Dims& d, const int32_t* nbr, void* ws, hipStream_t stream) {
    int* flag = reinterpret_cast<int*>(ws);
    int32_t* rslot = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(ws) + 256);
    hipLaunchKernelGGL(zero_flag_kernel, dim3(1), dim3(1), 0, stream, flag);
    const int64_t n = d.na * d.nb;
    const unsigned g = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(reverse_slot_kernel, dim3(g), dim3(256), 0, stream, d.na, d.nb, nbr, rslot, flag);
    return hipGetLastError();
}

hipError_t launch_combine_d(const Dims& d, const double* Dfull, const int32_t* nbr, double* Dc, void* ws,
                            hipStream_t stream) {
    const int32_t* rslot = reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(ws) + 256);
    const int64_t n = d.nqz * d.nw * d.na * d.nb * 9;
    const unsigned g = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL(combine_d_kernel, dim3(g), dim3(256), 0, stream, d, Dfull, nbr, rslot, Dc);
    return hipGetLastError();
}

}  // namespace sse
