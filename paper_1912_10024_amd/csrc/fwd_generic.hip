// Direct (term-by-term) forward kernel for shapes without a matrix-core
// specialisation.  One workgroup per output block Sigma[k,E,a]; every term of
// Eq. 3 is formed in fp64 on the vector ALUs as sum_i X_i . Y_i with
// X_i = grad_i H . G_b and Y_i = sum_j D_ij grad_j H_ba (the coefficients summed
// into the right factor first: 6 block products per term instead of 12), with
// grad_j H_ba the stored block B[a,n,j] when given, else grad_j H^H.
#include "sse_kernels.h"

namespace sse {

namespace {
constexpr int kGenThreads = 256;
constexpr int kGenMaxPerThread = 4;  // norb^2 <= 1024
}  // namespace

__global__ __launch_bounds__(kGenThreads) void fwd_generic_kernel(Dims d, const double* __restrict__ G,
                                                                  const double* __restrict__ Dp,
                                                                  const double* __restrict__ Dm,
                                                                  const double* __restrict__ A,
                                                                  const double* __restrict__ B,
                                                                  const int32_t* __restrict__ nbr, cd alpha,
                                                                  double* __restrict__ S) {
    extern __shared__ double smem[];
    const int N = (int)d.norb, NN = N * N;
    cd* sG = reinterpret_cast<cd*>(smem);  // [N][N]
    cd* sT = sG + NN;                      // [3][N][N]  X_i
    cd* sY = sT + 3 * NN;                  // [3][N][N]  Y_i
    const int tid = threadIdx.x;
    const int64_t nblk = d.nkz * d.ne * d.na;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t a = blk % d.na, e = (blk / d.na) % d.ne, k = blk / (d.na * d.ne);
        cd acc[kGenMaxPerThread];
#pragma unroll
        for (int x = 0; x < kGenMaxPerThread; ++x) acc[x] = cd{0.0, 0.0};
        for (int64_t q = 0; q < d.nqz; ++q) {
            const int64_t kp = ((k - q) % d.nkz + d.nkz) % d.nkz;
            for (int64_t w = 1; w <= d.nw; ++w) {
                for (int s = 1; s >= -1; s -= 2) {
                    const int64_t ep = e - s * w;
                    if (ep < 0 || ep >= d.ne) continue;
                    for (int64_t n = 0; n < d.nb; ++n) {
                        const int64_t b = nbr[a * d.nb + n];
                        if (b < 0 || b >= d.na) continue;
                        const double* Gb = G + 2 * off_G(d, kp, ep, b);
                        for (int x = tid; x < NN; x += kGenThreads) sG[x] = cload(Gb, x);
                        __syncthreads();
                        // G at E - w: coefficient at +w; G at E + w: coefficient at -w
                        const double* Dq = (s > 0 ? Dp : Dm) + 2 * off_D(d, q, w - 1, a, n);
                        for (int x = tid; x < 3 * NN; x += kGenThreads) {
                            const int i = x / NN, r = (x % NN) / N, u = x % N;
                            const double* Ai = A + 2 * off_A(d, a, n, i);
                            cd t = cd{0.0, 0.0};
                            for (int tt = 0; tt < N; ++tt) cfma(t, cload(Ai, r * N + tt), sG[tt * N + u]);
                            sT[x] = t;
                            // Y_i[r][u] = sum_j D_ij R_j[r][u], R_j = B_j or grad_j H^H
                            cd y = cd{0.0, 0.0};
                            for (int j = 0; j < 3; ++j) {
                                cd rj;
                                if (B) {
                                    rj = cload(B + 2 * off_A(d, a, n, j), r * N + u);
                                } else {
                                    const cd aj = cload(A + 2 * off_A(d, a, n, j), u * N + r);
                                    rj = cd{aj.re, -aj.im};
                                }
                                cfma(y, cload(Dq, i * 3 + j), rj);
                            }
                            sY[x] = y;
                        }
                        __syncthreads();
#pragma unroll
                        for (int xi = 0; xi < kGenMaxPerThread; ++xi) {
                            const int x = tid + xi * kGenThreads;
                            if (x >= NN) break;
                            const int r = x / N, c = x % N;
                            for (int i = 0; i < 3; ++i)
                                for (int uu = 0; uu < N; ++uu) cfma(acc[xi], sT[i * NN + r * N + uu], sY[i * NN + uu * N + c]);
                        }
                        __syncthreads();
                    }
                }
            }
        }
        double* Sb = S + 2 * off_S(d, k, e, a);
#pragma unroll
        for (int xi = 0; xi < kGenMaxPerThread; ++xi) {
            const int x = tid + xi * kGenThreads;
            if (x < NN) cstore(Sb, x, cmul(alpha, acc[xi]));
        }
    }
}

hipError_t launch_fwd_generic(const Dims& d, const double* G, const double* Dp, const double* Dm, const double* A,
                              const double* B, const int32_t* nbr, cd alpha, double* S, hipStream_t stream) {
    const int64_t nblk = d.nkz * d.ne * d.na;
    const unsigned grid = (unsigned)(nblk < (int64_t)(1 << 30) ? nblk : (1 << 30));
    const size_t lds = sizeof(cd) * 7 * (size_t)(d.norb * d.norb);  // G, X_i, Y_i
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fwd_generic_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fwd_generic_kernel, dim3(grid), dim3(kGenThreads), lds, stream, d, G, Dp, Dm, A, B, nbr, alpha, S);
    return hipGetLastError();
}

bool generic_supported(const Dims& d) { return d.norb * d.norb <= kGenThreads * kGenMaxPerThread; }

}  // namespace sse
