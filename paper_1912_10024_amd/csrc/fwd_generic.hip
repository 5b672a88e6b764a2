// Direct (term-by-term) forward kernel for shapes without a matrix-core
// specialisation.  One workgroup per output block Sigma[k,E,a]; every term of
// Eq. 3 is formed in fp64 on the vector ALUs as sum_i X_i . Y_i with
// X_i = grad_i H . G_b and Y_i = sum_j D_ij grad_j H_ba (the coefficients summed
// into the right factor first: 6 block products per term instead of 12), with
// grad_j H_ba the stored block B[a,n,j] when given, else grad_j H^H.
//
// The neighbour loop is outermost: a neighbour's left and right factors are
// staged in LDS once for all 2*Nqz*Nw of its terms (when they fit), and the
// G block of the next term is loaded while the current one is accumulated
// (two LDS buffers), so a term costs two barriers.  When Norb^2 is small, the
// sum over (i, u) of an output element is split over `parts` threads and
// reduced in LDS once per output block.
#include "sse_kernels.h"

namespace sse {

namespace {
constexpr int kGenThreads = 256;
constexpr int kGenMaxPerThread = 4;  // norb^2 <= 1024
constexpr int kGenMaxParts = 3;
// LDS (complex elements): G x2, X_i x3, Y_i x3, plus the staged factors x6
constexpr int kGenStageMaxNN = 292;  // 14 * NN * 16 B <= 64 KB

// number of threads that share one output element's sum
int gen_parts(int64_t nn) {
    const int64_t p = kGenThreads / nn;
    return (int)(p < 2 ? 1 : (p > kGenMaxParts ? kGenMaxParts : p));
}
}  // namespace

template <bool STAGE>
__global__ __launch_bounds__(kGenThreads) void fwd_generic_kernel(Dims d, const double* __restrict__ G,
                                                                  const double* __restrict__ Dp,
                                                                  const double* __restrict__ Dm,
                                                                  const double* __restrict__ A,
                                                                  const double* __restrict__ B,
                                                                  const int32_t* __restrict__ nbr, cd alpha,
                                                                  int parts, double* __restrict__ S) {
    extern __shared__ double smem[];
    const int N = (int)d.norb, NN = N * N;
    cd* sG = reinterpret_cast<cd*>(smem);  // [2][N][N]  G_b of this term and of the next
    cd* sT = sG + 2 * NN;                  // [3][N][N]  X_i (after the last term: the partial sums)
    cd* sY = sT + 3 * NN;                  // [3][N][N]  Y_i
    cd* sA = sY + 3 * NN;                  // [3][N][N]  grad_i H_ab          (STAGE)
    cd* sR = sA + 3 * NN;                  // [3][N][N]  right factor R_j     (STAGE)
    const int tid = threadIdx.x;
    const int64_t nblk = d.nkz * d.ne * d.na;
    const int64_t nterm = d.nqz * d.nw * 2;  // t -> (q, w, s): q = t / 2Nw, w = 1 + (t / 2) % Nw, s = +1 for even t
    const int nitems = parts * NN;           // parts > 1 only when parts * NN <= kGenThreads
    const int span = 3 * N;                  // the (i, u) sum of one output element
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t a = blk % d.na, e = (blk / d.na) % d.ne, k = blk / (d.na * d.ne);
        // the G block term t reads, or nterm when no later term is inside the energy grid
        auto next_valid = [&](int64_t t) {
            for (; t < nterm; ++t) {
                const int64_t w = 1 + (t / 2) % d.nw, ep = e - ((t & 1) ? -w : w);
                if (ep >= 0 && ep < d.ne) break;
            }
            return t;
        };
        auto load_g = [&](int64_t t, int64_t b, cd* dst) {
            const int64_t q = t / (2 * d.nw), w = 1 + (t / 2) % d.nw, ep = e - ((t & 1) ? -w : w);
            const int64_t kp = ((k - q) % d.nkz + d.nkz) % d.nkz;
            const double* Gb = G + 2 * off_G(d, kp, ep, b);
            for (int x = tid; x < NN; x += kGenThreads) dst[x] = cload(Gb, x);
        };
        cd acc[kGenMaxPerThread];
#pragma unroll
        for (int x = 0; x < kGenMaxPerThread; ++x) acc[x] = cd{0.0, 0.0};
        for (int64_t n = 0; n < d.nb; ++n) {
            const int64_t b = nbr[a * d.nb + n];
            if (b < 0 || b >= d.na) continue;
            if constexpr (STAGE) {
                for (int x = tid; x < 3 * NN; x += kGenThreads) {
                    const int i = x / NN, r = (x % NN) / N, u = x % N;
                    sA[x] = cload(A + 2 * off_A(d, a, n, i), r * N + u);
                    if (B) {
                        sR[x] = cload(B + 2 * off_A(d, a, n, i), r * N + u);
                    } else {
                        const cd aj = cload(A + 2 * off_A(d, a, n, i), u * N + r);
                        sR[x] = cd{aj.re, -aj.im};
                    }
                }
            }
            int64_t t = next_valid(0);
            if (t < nterm) load_g(t, b, sG);
            __syncthreads();
            int buf = 0;
            while (t < nterm) {
                const cd* sGc = sG + buf * NN;
                const int64_t q = t / (2 * d.nw), w = 1 + (t / 2) % d.nw;
                // G at E - w: coefficient at +w; G at E + w: coefficient at -w
                const double* Dq = ((t & 1) ? Dm : Dp) + 2 * off_D(d, q, w - 1, a, n);
                for (int x = tid; x < 3 * NN; x += kGenThreads) {
                    const int i = x / NN, r = (x % NN) / N, u = x % N;
                    cd tx = cd{0.0, 0.0};
                    cd y = cd{0.0, 0.0};
                    if constexpr (STAGE) {
                        const cd* Ai = sA + i * NN + r * N;
                        for (int tt = 0; tt < N; ++tt) cfma(tx, Ai[tt], sGc[tt * N + u]);
                        for (int j = 0; j < 3; ++j) cfma(y, cload(Dq, i * 3 + j), sR[j * NN + r * N + u]);
                    } else {
                        const double* Ai = A + 2 * off_A(d, a, n, i);
                        for (int tt = 0; tt < N; ++tt) cfma(tx, cload(Ai, r * N + tt), sGc[tt * N + u]);
                        // Y_i[r][u] = sum_j D_ij R_j[r][u], R_j = B_j or grad_j H^H
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
                    }
                    sT[x] = tx;
                    sY[x] = y;
                }
                __syncthreads();
                const int64_t tn = next_valid(t + 1);
                if (tn < nterm) load_g(tn, b, sG + (buf ^ 1) * NN);
#pragma unroll
                for (int xi = 0; xi < kGenMaxPerThread; ++xi) {
                    const int it = tid + xi * kGenThreads;
                    if (it >= nitems) break;
                    const int x = it % NN, p = it / NN;
                    const int r = x / N, col = x % N;
                    const int c0 = p * span / parts, c1 = (p + 1) * span / parts;
                    int i = c0 / N, uu = c0 % N;
                    for (int c = c0; c < c1; ++c) {
                        cfma(acc[xi], sT[i * NN + r * N + uu], sY[i * NN + uu * N + col]);
                        if (++uu == N) {
                            uu = 0;
                            ++i;
                        }
                    }
                }
                __syncthreads();
                t = tn;
                buf ^= 1;
            }
        }
        double* Sb = S + 2 * off_S(d, k, e, a);
        if (parts == 1) {
#pragma unroll
            for (int xi = 0; xi < kGenMaxPerThread; ++xi) {
                const int x = tid + xi * kGenThreads;
                if (x < NN) cstore(Sb, x, cmul(alpha, acc[xi]));
            }
        } else {
            // one item per thread: partial p of element x at sT[p * NN + x]
            __syncthreads();
            if (tid < nitems) sT[tid] = acc[0];
            __syncthreads();
            if (tid < NN) {
                cd s = sT[tid];
                for (int p = 1; p < parts; ++p) {
                    const cd v = sT[p * NN + tid];
                    s.re += v.re;
                    s.im += v.im;
                }
                cstore(Sb, tid, cmul(alpha, s));
            }
            __syncthreads();
        }
    }
}

hipError_t launch_fwd_generic(const Dims& d, const double* G, const double* Dp, const double* Dm, const double* A,
                              const double* B, const int32_t* nbr, cd alpha, double* S, hipStream_t stream) {
    const int64_t nblk = d.nkz * d.ne * d.na;
    const unsigned grid = (unsigned)(nblk < (int64_t)(1 << 30) ? nblk : (1 << 30));
    const int64_t nn = d.norb * d.norb;
    const int parts = gen_parts(nn);
    const bool stage = nn <= kGenStageMaxNN;
    const size_t lds = sizeof(cd) * (stage ? 14 : 8) * (size_t)nn;  // G x2, X_i, Y_i (+ staged factors)
    const void* kern = stage ? reinterpret_cast<const void*>(fwd_generic_kernel<true>)
                             : reinterpret_cast<const void*>(fwd_generic_kernel<false>);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (stage)
        hipLaunchKernelGGL(fwd_generic_kernel<true>, dim3(grid), dim3(kGenThreads), lds, stream, d, G, Dp, Dm, A, B,
                           nbr, alpha, parts, S);
    else
        hipLaunchKernelGGL(fwd_generic_kernel<false>, dim3(grid), dim3(kGenThreads), lds, stream, d, G, Dp, Dm, A, B,
                           nbr, alpha, parts, S);
    return hipGetLastError();
}

bool generic_supported(const Dims& d) { return d.norb * d.norb <= kGenThreads * kGenMaxPerThread; }

}  // namespace sse
