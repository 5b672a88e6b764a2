// Phonon scattering self-energy (Eq. 4) for the off-diagonal blocks kept per
// atom pair (a, b = nbr[a, n]), where the sum over l reduces to l = b:
//
//   Pi[q, w-1, a, n][i][j] = beta * sum_k sum_{E : E + w < NE}
//       tr( A_i^H . Gs[(k+q) mod Nkz, E+w, a] . A_j . Go[k, E, b] ),   A_i = grad_i H_ab
//
// By the cyclic property of the trace, tr(A_i^H Gs A_j Go) = sum_{s,t} Gs[s][t] T_ij[t][s]
// with T_ij = A_j . Go . A_i^H.  T is formed once per source point (k, E) and
// neighbour slot, and reused by all Nqz * Nw shifted Gs blocks it meets (the
// same fission the paper applies to Eq. 3, Sec. "Dataflow Optimizations").
//
// pse_mfma_kernel (Norb 10, Nkz 7, Nw 10, NB 4): one workgroup of 8 waves per
// atom a sweeps the source points (E outer, k inner).  Per source point:
//   1. V[n][j] = A_j . Go[k, E, nbr[a,n]]          (fp64 VALU, LDS)
//   2. T[n][i][j] = V[n][j] . A_i^H                 (fp64 VALU, into two LDS planes)
//   3. C[(q,w), (n,i,j,re/im)] += sum over (s,t,re/im) of
//        Gs[(k+q) mod Nkz, E+w, a][s][t] (re or im) * B[(s,t,re/im), (n,i,j,re/im)]
//      on the fp64 matrix cores: M = Nkz Nw = 70 rows (5 tiles), N = 2 * 9 NB = 72
//      columns (5 tiles), K = 2 Norb^2 = 200 (50 k-steps).  B is the real
//      embedding [[Tr, Ti], [-Ti, Tr]] of T; the A rows are read straight from Gs
//      in global memory (one row = one Gs block, reused by the column tiles).
//      The waves form 4 K groups (k-steps dealt round-robin) x 2 tile groups
//      (13 and 12 of the 25 tiles), so the two waves on a SIMD share its matrix
//      core and each hides the other's load and barrier waits.
// Two barriers per source point: Go is double-buffered in LDS and prefetched
// two points ahead in registers.  After the sweep the K groups' accumulators
// are added in a fixed order in LDS, scaled by beta and written out; every
// output entry is written once.
//
// pse_generic_kernel (any other shape): one workgroup per neighbour slot, the
// same three steps on the vector ALUs with one thread per (q, w).
#include "sse_kernels.h"

namespace sse {

typedef double pse_f64x4 __attribute__((ext_vector_type(4)));

// A zero Gs block: read by the padding rows of the GEMM and by rows whose
// energy E + w leaves the grid, so the row loads need no branch.
__device__ const double pse_zero_block[256] = {};

template <int N, int NK, int NW, int NB>
struct PseCfg {
    static constexpr int KG = 4;                       // K groups: k-steps kg, kg + KG, ...
    static constexpr int TG = 2;                       // tile groups
    static constexpr int WAVES = KG * TG, THREADS = 64 * WAVES;
    static constexpr int NN = N * N;
    static constexpr int NCOLC = 9 * NB;               // complex GEMM columns (n, i, j)
    static constexpr int NT = (2 * NCOLC + 15) / 16;   // column tiles
    static constexpr int CPAD = 8 * NT;                // complex columns per T plane row, with padding
    static constexpr int MROWS = NK * NW;              // (q, w) rows
    static constexpr int MT = (MROWS + 15) / 16;       // row tiles
    static constexpr int NTILES = MT * NT;
    static constexpr int SL = (NTILES + 1) / 2;        // tiles (accumulator slots) of tile group 0
    static constexpr int ML = (SL + NT - 1) / NT;      // row tiles a wave touches
    static constexpr int KSTEPS = NN / 2;              // 2 Norb^2 real K rows, 4 per k-step
    static constexpr int KS_MAX = (KSTEPS + KG - 1) / KG;
    // the im plane starts 8 doubles (16 LDS banks) past a multiple of the re
    // plane size, so a 16-lane group reading 8 columns of each plane is conflict-free
    static constexpr int PLANE = NN * CPAD + 8;
    static constexpr int L_A = NB * 3 * NN * 2;        // grad H of the atom (doubles)
    static constexpr int L_GO = 2 * NB * NN * 2;       // Go blocks, double-buffered
    static constexpr int L_V = NB * 3 * NN * 2;        // V = A_j Go
    static constexpr int L_T = 2 * PLANE;              // T planes (re, im)
    static constexpr int L_RED = KG * NT * 256;        // reduction scratch, aliases the T planes
    static constexpr int L_TR = L_T > L_RED ? L_T : L_RED;
    static constexpr size_t LDS_BYTES = sizeof(double) * (L_A + L_GO + L_V + L_TR);
    static_assert(NN % 2 == 0, "K = 2 Norb^2 must split into k-steps of 4");
    static_assert(2 * NN <= 256, "zero block too small");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(NB * N * N <= THREADS, "formation tasks: at most one per thread");
    static_assert(NTILES - SL <= SL && ML <= MT, "tile groups");
};

// Tile of accumulator slot s: group 0 holds tiles 0 .. SL-1 in row-major
// order, group 1 the rest counted from the last tile backwards, so both
// groups run the same slot schedule with mirrored tile indices.
template <class C>
__device__ __forceinline__ int pse_tile_mt(int tg, int s) { return tg ? C::MT - 1 - s / C::NT : s / C::NT; }
template <class C>
__device__ __forceinline__ int pse_tile_nt(int tg, int s) { return tg ? C::NT - 1 - s % C::NT : s % C::NT; }

template <int N, int NK, int NW, int NB>
__global__ __launch_bounds__(512) void pse_mfma_kernel(Dims d, const double* __restrict__ Gs,
                                                       const double* __restrict__ Go, const double* __restrict__ Ag,
                                                       const int32_t* __restrict__ nbr, cd beta,
                                                       double* __restrict__ Pi) {
    using C = PseCfg<N, NK, NW, NB>;
    constexpr int NN = C::NN;
    extern __shared__ __align__(16) double smem[];
    double* sA = smem;           // [NB][3][N][N] complex
    double* sGo = sA + C::L_A;   // [2][NB][N][N] complex
    double* sV = sGo + C::L_GO;  // [NB][3 (j)][N (t)][N (r)] complex
    double* sT = sV + C::L_V;    // re plane [NN][CPAD], im plane at +PLANE; entry (s*N + t, n*9 + i*3 + j) = T_ij[t][s]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kg = wave % C::KG, tg = wave / C::KG;
    const int64_t a = blockIdx.x;
    const int NE = (int)d.ne;
    const int64_t NA = d.na;
    const int64_t slot = 2 * d.gs * NN;   // doubles between atoms at one (k, E)
    const int64_t e_step = slot * NA;      // doubles between energies
    const int64_t k_step = e_step * NE;    // doubles between momenta

    for (int x = tid; x < NB * 3 * NN; x += C::THREADS) {
        const cd v = cload(Ag, off_A(d, a, 0, 0) + x);
        sA[2 * x] = v.re;
        sA[2 * x + 1] = v.im;
    }
    for (int x = tid; x < C::L_TR; x += C::THREADS) sT[x] = 0.0;

    // Go: thread tid < NB*NN moves complex element tid of the NB blocks
    const bool go_lane = tid < NB * NN;
    int64_t go_off;
    bool go_ok;
    {
        const int32_t b = go_lane ? nbr[a * NB + tid / NN] : -1;
        go_ok = b >= 0 && b < NA;
        go_off = go_ok ? slot * b + 2 * (tid % NN) : 0;
    }
    cd gov;
    auto load_go = [&](int src) {
        const int E = src / NK, k = src % NK;
        const double* p = go_ok ? Go + k * k_step + (int64_t)E * e_step + go_off : pse_zero_block;
        const double2 v = *reinterpret_cast<const double2*>(p);
        gov = cd{v.x, v.y};
    };
    auto store_go = [&](int src) {
        if (go_lane) *reinterpret_cast<double2*>(sGo + (src & 1) * (NB * NN * 2) + 2 * tid) = make_double2(gov.re, gov.im);
    };

    // GEMM operand lanes.  A (16 x 4 per k-step): lane holds row j16, K index kk;
    // B (4 x 16): K index kk, column j16.  K index 4 ks + kk = (Gs element
    // s*N + t = 2 ks + kk/2, re/im = kk & 1).
    const int kk = lane >> 4, j16 = lane & 15, kc = kk & 1;
    int a_q[C::ML], a_w[C::ML];
    bool a_row[C::ML];
#pragma unroll
    for (int ml = 0; ml < C::ML; ++ml) {
        const int mt = tg ? C::MT - 1 - ml : ml;
        const int r = 16 * mt + j16;
        a_row[ml] = r < C::MROWS;
        a_q[ml] = r / NW;
        a_w[ml] = r % NW + 1;
    }
    // B: plane (re or im) and sign of this lane's entry of [[Tr, Ti], [-Ti, Tr]]
    const double* bp[C::NT];
    long long b_neg;
    {
        const int dd = j16 & 1;
        const int plane = (kc ^ dd) ? C::PLANE : 0;
        b_neg = (kc == 1 && dd == 0) ? (long long)0x8000000000000000ull : 0ll;
#pragma unroll
        for (int nl = 0; nl < C::NT; ++nl) {
            const int nt = tg ? C::NT - 1 - nl : nl;
            bp[nl] = sT + plane + (kk >> 1) * C::CPAD + 8 * nt + (j16 >> 1) + 2 * kg * C::CPAD;
        }
    }
    const bool last_slot = tg == 0;   // group 0 owns one tile more when NTILES is odd

    pse_f64x4 acc[C::SL];
#pragma unroll
    for (int s = 0; s < C::SL; ++s) acc[s] = pse_f64x4{0.0, 0.0, 0.0, 0.0};

    const int nsrc = NK * NE;
    load_go(0);
    store_go(0);
    if (nsrc > 1) load_go(1);
    __syncthreads();
    for (int src = 0; src < nsrc; ++src) {
        const int E = src / NK, k = src % NK;
        // 1. V[n][j][t][r] = sum_u A[n][j][t][u] Go[n][u][r], three j per task
        if (tid < NB * NN) {
            const int n = tid / NN, t = (tid / N) % N, r = tid % N;
            const double* A0 = sA + 2 * ((n * 3) * NN + t * N);
            const double* G0 = sGo + (src & 1) * (NB * NN * 2) + 2 * (n * NN + r);
            cd v0{0.0, 0.0}, v1{0.0, 0.0}, v2{0.0, 0.0};
#pragma unroll
            for (int u = 0; u < N; ++u) {
                const cd g{G0[2 * u * N], G0[2 * u * N + 1]};
                cfma(v0, cd{A0[2 * u], A0[2 * u + 1]}, g);
                cfma(v1, cd{A0[2 * (NN + u)], A0[2 * (NN + u) + 1]}, g);
                cfma(v2, cd{A0[2 * (2 * NN + u)], A0[2 * (2 * NN + u) + 1]}, g);
            }
            double* V0 = sV + 2 * ((n * 3) * NN + t * N + r);
            *reinterpret_cast<double2*>(V0) = make_double2(v0.re, v0.im);
            *reinterpret_cast<double2*>(V0 + 2 * NN) = make_double2(v1.re, v1.im);
            *reinterpret_cast<double2*>(V0 + 4 * NN) = make_double2(v2.re, v2.im);
        }
        __syncthreads();   // V complete; every wave is past the previous contraction
        // 2. T[n][i][j][t][s] = sum_r V[n][j][t][r] conj(A[n][i][s][r]), nine (i, j) per task
        if (tid < NB * NN) {
            const int n = tid / NN, t = (tid / N) % N, s = tid % N;
            const double* V0 = sV + 2 * ((n * 3) * NN + t * N);
            const double* A0 = sA + 2 * ((n * 3) * NN + s * N);
            cd tv[9];
#pragma unroll
            for (int ij = 0; ij < 9; ++ij) tv[ij] = cd{0.0, 0.0};
#pragma unroll
            for (int r = 0; r < N; ++r) {
                cd vj[3], ai[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    vj[m] = cd{V0[2 * (m * NN + r)], V0[2 * (m * NN + r) + 1]};
                    ai[m] = cd{A0[2 * (m * NN + r)], A0[2 * (m * NN + r) + 1]};
                }
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) cfma_conj(tv[i * 3 + j], vj[j], ai[i]);
            }
            double* T0 = sT + (s * N + t) * C::CPAD + n * 9;
#pragma unroll
            for (int ij = 0; ij < 9; ++ij) {
                T0[ij] = tv[ij].re;
                T0[C::PLANE + ij] = tv[ij].im;
            }
        }
        // Go of the next source point into the free buffer, the one after that into registers
        if (src + 1 < nsrc) store_go(src + 1);
        if (src + 2 < nsrc) load_go(src + 2);
        // A row bases of this source point (the wave's first k-step and the lane's K index
        // folded in) and the first k-step's rows
        const double* ap[C::ML];
#pragma unroll
        for (int ml = 0; ml < C::ML; ++ml) {
            const int es = E + a_w[ml];
            const bool ok = a_row[ml] && es < NE;
            const int kq = (k + a_q[ml]) % NK;
            const double* p = ok ? Gs + kq * k_step + (int64_t)es * e_step + slot * a : pse_zero_block;
            ap[ml] = p + 4 * kg + kk;
        }
        double an[C::ML];
#pragma unroll
        for (int ml = 0; ml < C::ML; ++ml) an[ml] = ap[ml][0];
        __syncthreads();   // T complete
        // 3. the contraction on the matrix cores: k-steps kg, kg + KG, ...
#pragma unroll
        for (int i = 0; i < C::KS_MAX; ++i) {
            const bool live = kg + C::KG * i < C::KSTEPS;
            double ac[C::ML];
#pragma unroll
            for (int ml = 0; ml < C::ML; ++ml) ac[ml] = an[ml];
            if (i + 1 < C::KS_MAX && kg + C::KG * (i + 1) < C::KSTEPS) {
#pragma unroll
                for (int ml = 0; ml < C::ML; ++ml) an[ml] = ap[ml][4 * C::KG * (i + 1)];
            }
            if (live) {
                double bv[C::NT];
#pragma unroll
                for (int nl = 0; nl < C::NT; ++nl)
                    bv[nl] = __longlong_as_double(__double_as_longlong(bp[nl][2 * C::KG * i * C::CPAD]) ^ b_neg);
#pragma unroll
                for (int s = 0; s < C::SL; ++s) {
                    if (s == C::SL - 1 && C::SL * 2 != C::NTILES && !last_slot) continue;
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[s / C::NT], bv[s % C::NT], acc[s], 0, 0, 0);
                }
            }
        }
    }

    // Sum of the K groups' partial results in K-group order, scaled by beta.
    __syncthreads();
    double* red = sT;   // [KG][NT][16 rows][16 cols]
    for (int mt = 0; mt < C::MT; ++mt) {
#pragma unroll
        for (int s = 0; s < C::SL; ++s) {
            if (s == C::SL - 1 && C::SL * 2 != C::NTILES && !last_slot) continue;
            if (pse_tile_mt<C>(tg, s) != mt) continue;
            const int nt = pse_tile_nt<C>(tg, s);
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(kg * C::NT + nt) * 256 + (4 * v + (lane >> 4)) * 16 + j16] = acc[s][v];
        }
        __syncthreads();
        for (int x = tid; x < C::NT * 16 * 8; x += C::THREADS) {
            const int nt = x / 128, row = (x / 8) % 16, cp = x % 8;
            const int rg = 16 * mt + row, colc = 8 * nt + cp;
            if (rg < C::MROWS && colc < C::NCOLC) {
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int g = 0; g < C::KG; ++g) {
                    const double* p = red + (g * C::NT + nt) * 256 + row * 16 + 2 * cp;
                    re += p[0];
                    im += p[1];
                }
                const int q = rg / NW, wi = rg % NW, n = colc / 9, ij = colc % 9;
                cstore(Pi, off_D(d, q, wi, a, n) + ij, cmul(beta, cd{re, im}));
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ generic
constexpr int kPseThreads = 256;

__global__ __launch_bounds__(kPseThreads) void pse_generic_kernel(Dims d, const double* __restrict__ Gs,
                                                                  const double* __restrict__ Go,
                                                                  const double* __restrict__ Ag,
                                                                  const int32_t* __restrict__ nbr, cd beta,
                                                                  double* __restrict__ Pi) {
    extern __shared__ __align__(16) double smem[];
    const int N = (int)d.norb, NN = N * N;
    const int nqw = (int)(d.nqz * d.nw);
    cd* sA = reinterpret_cast<cd*>(smem);  // [3][N][N]
    cd* sG = sA + 3 * NN;                  // [N][N]   Go block of the source point
    cd* sV = sG + NN;                      // [3][N][N] V_j = A_j Go
    cd* sT = sV + 3 * NN;                  // [9][NN]  entry (ij, s*N + t) = T_ij[t][s]
    const int tid = threadIdx.x;
    const int64_t edge = blockIdx.x;
    const int64_t a = edge / d.nb, n = edge % d.nb;
    const int32_t b = nbr[edge];
    const bool valid_b = b >= 0 && b < d.na;
    for (int x = tid; x < 3 * NN; x += kPseThreads) sA[x] = cload(Ag, off_A(d, a, n, 0) + x);
    constexpr int kPer = 2;
    cd acc[kPer][9];
#pragma unroll
    for (int s = 0; s < kPer; ++s)
#pragma unroll
        for (int ij = 0; ij < 9; ++ij) acc[s][ij] = cd{0.0, 0.0};
    for (int64_t k = 0; k < d.nkz; ++k)
        for (int64_t e = 0; e < d.ne; ++e) {
            __syncthreads();
            for (int x = tid; x < NN; x += kPseThreads) sG[x] = valid_b ? cload(Go, off_G(d, k, e, b) + x) : cd{0.0, 0.0};
            __syncthreads();
            for (int x = tid; x < 3 * NN; x += kPseThreads) {
                const int j = x / NN, t = (x % NN) / N, r = x % N;
                cd s{0.0, 0.0};
                for (int u = 0; u < N; ++u) cfma(s, sA[j * NN + t * N + u], sG[u * N + r]);
                sV[x] = s;
            }
            __syncthreads();
            for (int x = tid; x < 9 * NN; x += kPseThreads) {
                const int ij = x / NN, i = ij / 3, j = ij % 3, kap = x % NN, s_ = kap / N, t = kap % N;
                cd s{0.0, 0.0};
                for (int r = 0; r < N; ++r) cfma_conj(s, sV[j * NN + t * N + r], sA[i * NN + s_ * N + r]);
                sT[x] = s;
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                const int qw = tid + s * kPseThreads;
                if (qw < nqw) {
                    const int64_t q = qw / d.nw, w = qw % d.nw + 1;
                    if (e + w < d.ne) {
                        const int64_t g0 = off_G(d, (k + q) % d.nkz, e + w, a);
                        for (int kap = 0; kap < NN; ++kap) {
                            const cd gv = cload(Gs, g0 + kap);
#pragma unroll
                            for (int ij = 0; ij < 9; ++ij) cfma(acc[s][ij], gv, sT[ij * NN + kap]);
                        }
                    }
                }
            }
        }
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
        const int qw = tid + s * kPseThreads;
        if (qw < nqw) {
            const int64_t q = qw / d.nw, w = qw % d.nw;
#pragma unroll
            for (int ij = 0; ij < 9; ++ij) cstore(Pi, off_D(d, q, w, a, n) + ij, cmul(beta, acc[s][ij]));
        }
    }
}

static size_t pse_generic_lds(const Dims& d) {
    return sizeof(cd) * 16 * (size_t)(d.norb * d.norb);
}

bool pse_mfma_specialised(const Dims& d) {
    return d.norb == 10 && d.nkz == 7 && d.nqz == 7 && d.nw == 10 && d.nb == 4 && d.ne < (1 << 28);
}

bool pse_generic_supported(const Dims& d) {
    return d.nqz * d.nw <= 2 * kPseThreads && pse_generic_lds(d) <= 160 * 1024 && d.na * d.nb <= INT32_MAX;
}

hipError_t launch_pse(const Dims& d, const double* Gs, const double* Go, const double* A, const int32_t* nbr, cd beta,
                      double* Pi, hipStream_t stream) {
    if (pse_mfma_specialised(d)) {
        using C = PseCfg<10, 7, 10, 4>;
        auto kern = pse_mfma_kernel<10, 7, 10, 4>;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS_BYTES);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3((unsigned)d.na), dim3(C::THREADS), C::LDS_BYTES, stream, d, Gs, Go, A, nbr, beta,
                           Pi);
        return hipGetLastError();
    }
    const size_t lds = pse_generic_lds(d);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(pse_generic_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pse_generic_kernel, dim3((unsigned)(d.na * d.nb)), dim3(kPseThreads), lds, stream, d, Gs, Go, A,
                       nbr, beta, Pi);
    return hipGetLastError();
}

}  // namespace sse
