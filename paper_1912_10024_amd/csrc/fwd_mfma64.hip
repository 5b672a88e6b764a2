// FP64 matrix-core forward kernel of the scattering self-energy (Eq. 3).
//
// Regrouping (the fission of Sec. "Dataflow Optimizations", taken one step
// further so the matrix cores see one dense GEMM per atom):
//
//   P[k',E',n,i,j] = grad_i H_{a,n} . G[k',E',nbr[a,n],0] . grad_j H_{a,n}^H     (Norb x Norb)
//   V[(k,w),(E',r,c)] = sum_{k',n,i,j} D[(k-k') mod Nkz, w-1, a, n, i, j] * P[k',E',n,i,j][r,c]
//   Sigma[k,E,a][r,c] = alpha * sum_w ( V[(k,w),(E-w,r,c)] + V[(k,w),(E+w,r,c)] )
//
// The momentum convolution (sum over qz with k' = k - qz) sits inside the
// GEMM's K dimension: the D operand is the circulant block matrix
// D[(k - k') mod Nkz], built on the fly from a per-atom table in LDS.  The
// energy convolution (w, +/-) is the stencil applied to the GEMM output.
//
// Work decomposition: one workgroup of 8 waves per (atom a, output row r);
// it sweeps the energy axis in blocks of EB source energies.  Per block the
// GEMM is M = 2*Nkz*Nw real rows (k, w, re/im), N = EB*Norb columns (E', c),
// K = Nkz * Nb * 9 complex, consumed in chunks of one k' and two neighbours
// (36 real K rows = 9 MFMA k-steps).  Complex products use the real
// embedding [[Dr, -Di], [Di, Dr]] . [Pr; Pi].
//
// Pipeline per chunk (one barrier): every wave issues its share of the
// 16x16x4 fp64 MFMAs on the P chunk in LDS, forms the next P chunk from the
// X = grad_i H . G rows of the chunk after (vector ALUs, double-buffered
// in LDS), and gathers the G blocks for the chunk after that from HBM.  The
// waves on one SIMD alternate which of the two they do first, so one wave's
// vector work runs under the other's matrix instructions.  At the end of an
// energy block each wave adds its accumulators into a ring of output planes
// (LDS, fp64), in wave order so that results are bitwise reproducible;
// planes that can receive no more contributions are scaled by alpha and
// written out.
#include "sse_kernels.h"

namespace sse {

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int NORB, int NKZ, int NW, int NB, int EB>
struct Fwd64 {
    static constexpr int WAVES = 8, THREADS = 64 * WAVES;
    static constexpr int MROWS = 2 * NKZ * NW;
    static constexpr int MT = (MROWS + 15) / 16;
    static constexpr int NCOLS = EB * NORB;
    static constexpr int NT = (NCOLS + 15) / 16;
    static constexpr int NCP = NT * 16;
    static constexpr int NPAIR = MT * NT;
    static constexpr int PPW = (NPAIR + WAVES - 1) / WAVES;
    static constexpr int NP = (NB + 1) / 2;
    static constexpr int NCHUNK = NKZ * NP;
    static constexpr int KR = 36;
    static constexpr int KS = 9;
    static constexpr int RING = EB + 2 * NW;
    static constexpr int WS = NB * 18 + 2;  // padded D-table stride per w (bank spread)
    static constexpr int QS = NW * WS;
    static constexpr int NN = NORB * NORB;
    // LDS carve-up, in doubles
    static constexpr int L_D = NKZ * QS;
    static constexpr int L_A = NB * 3 * NN * 2;
    static constexpr int L_P = 2 * KR * NCP;
    static constexpr int XB = EB * 2 * 3 * NORB * 2;  // one X buffer: [el][nl][i][u] complex
    static constexpr int L_X = 2 * XB;
    static constexpr int RP = NKZ * NORB * 2;  // one ring plane: [k][c] complex
    static constexpr int L_R = RING * RP;
    static constexpr size_t LDS_BYTES = sizeof(double) * (size_t)(L_D + L_A + L_P + L_X + L_R);
    static constexpr int X_ITEMS = EB * 2 * 3 * NORB;
    static constexpr int X_IPW = (X_ITEMS + WAVES - 1) / WAVES;
    static constexpr int P_ITEMS = EB * 2 * NORB;
    static constexpr int P_IPW = (P_ITEMS + WAVES - 1) / WAVES;
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(X_IPW <= 64 && P_IPW <= 64, "one item per lane");
    static_assert(PPW <= MT + 1, "a wave's pairs span at most two N-tiles");
};

template <int NORB, int NKZ, int NW, int NB, int EB>
__global__ __launch_bounds__(512) void fwd_mfma64_kernel(Dims d, const double* __restrict__ G,
                                                         const double* __restrict__ Dg,
                                                         const double* __restrict__ Ag,
                                                         const int32_t* __restrict__ nbr, cd alpha,
                                                         double* __restrict__ S) {
    using C = Fwd64<NORB, NKZ, NW, NB, EB>;
    extern __shared__ double lds[];
    double* sD = lds;
    double* sA = sD + C::L_D;
    double* sP = sA + C::L_A;
    double* sX = sP + C::L_P;
    double* sR = sX + C::L_X;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // XCD-aware mapping: the Norb workgroups of one atom share its D, grad H and
    // neighbour G blocks, so they get block ids that land on the same XCD.
    const int64_t bid = blockIdx.x;
    const int r = (int)((bid >> 3) % NORB);
    const int64_t a = ((bid >> 3) / NORB) * 8 + (bid & 7);
    if (a >= d.na) return;  // uniform for the whole workgroup, before any barrier

    // ---- stage the atom's D table, grad H and the neighbour list; clear buffers
    for (int x = tid; x < NKZ * NW * NB * 9; x += C::THREADS) {
        const int ij = x % 9, n = (x / 9) % NB, w = (x / (9 * NB)) % NW, q = x / (9 * NB * NW);
        const cd v = cload(Dg, off_D(d, q, w, a, n) + ij);
        sD[q * C::QS + w * C::WS + n * 18 + ij * 2] = v.re;
        sD[q * C::QS + w * C::WS + n * 18 + ij * 2 + 1] = v.im;
    }
    for (int x = tid; x < NB * 3 * C::NN; x += C::THREADS) {
        const cd v = cload(Ag, off_A(d, a, 0, 0) + x);
        sA[2 * x] = v.re;
        sA[2 * x + 1] = v.im;
    }
    for (int x = tid; x < C::L_P; x += C::THREADS) sP[x] = 0.0;
    for (int x = tid; x < C::L_R; x += C::THREADS) sR[x] = 0.0;
    int32_t nb_atom[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) nb_atom[n] = nbr[a * NB + n];

    const int64_t NE = d.ne;
    const int64_t nblk = (NE + EB - 1) / EB;
    const int64_t niter = nblk * C::NCHUNK;

    // ---- X rows: X[el][nl][i][u] = sum_t gradH[n][i][r][t] G[k'][e0+el][b][t][u]
    auto produce_x = [&](int64_t g) {
        if (g >= niter) return;
        const int64_t blk = g / C::NCHUNK;
        const int ch = (int)(g % C::NCHUNK), kp = ch / C::NP, np = ch % C::NP;
        double* X = sX + (g & 1) * C::XB;
        const int item = wave * C::X_IPW + lane;
        if (lane < C::X_IPW && item < C::X_ITEMS) {
            const int u = item % NORB, i = (item / NORB) % 3, nl = (item / (3 * NORB)) % 2, el = item / (6 * NORB);
            const int n = 2 * np + nl;
            const int64_t e = blk * EB + el;
            cd acc{0.0, 0.0};
            if (n < NB && e < NE) {
                const int32_t b = nb_atom[n < NB ? n : 0];
                if (b >= 0 && b < d.na) {
                    const double* Gb = G + 2 * off_G(d, kp, e, b);
                    const double* Ar = sA + 2 * ((n * 3 + i) * C::NN + r * NORB);
#pragma unroll
                    for (int t = 0; t < NORB; ++t) {
                        const cd gv = cload(Gb, t * NORB + u);
                        cfma(acc, cd{Ar[2 * t], Ar[2 * t + 1]}, gv);
                    }
                }
            }
            X[2 * item] = acc.re;
            X[2 * item + 1] = acc.im;
        }
    };

    // ---- P chunk: P[(nl,i,j,re/im)][(el,c)] = sum_u X[el][nl][i][u] conj(gradH[n][j][c][u])
    auto produce_p = [&](int64_t g) {
        if (g >= niter) return;
        const int ch = (int)(g % C::NCHUNK), np = ch % C::NP;
        const double* X = sX + (g & 1) * C::XB;
        double* P = sP + (g & 1) * (C::KR * C::NCP);
        const int item = wave * C::P_IPW + lane;
        if (lane < C::P_IPW && item < C::P_ITEMS) {
            const int c = item % NORB, nl = (item / NORB) % 2, el = item / (2 * NORB);
            const int n = 2 * np + nl;
            const int col = el * NORB + c;
            if (n < NB) {
                const double* Xe = X + 2 * ((el * 2 + nl) * 3) * NORB;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double* Ac = sA + 2 * ((n * 3 + j) * C::NN + c * NORB);
                    cd ac[NORB];
#pragma unroll
                    for (int u = 0; u < NORB; ++u) ac[u] = cd{Ac[2 * u], Ac[2 * u + 1]};
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        cd p{0.0, 0.0};
#pragma unroll
                        for (int u = 0; u < NORB; ++u) cfma_conj(p, cd{Xe[2 * (i * NORB + u)], Xe[2 * (i * NORB + u) + 1]}, ac[u]);
                        const int kr = ((nl * 3 + i) * 3 + j) * 2;
                        P[kr * C::NCP + col] = p.re;
                        P[(kr + 1) * C::NCP + col] = p.im;
                    }
                }
            } else {
#pragma unroll
                for (int kr = nl * 18; kr < nl * 18 + 18; ++kr) P[kr * C::NCP + col] = 0.0;
            }
        }
    };

    // ---- this wave's (M-tile, N-tile) pairs, N-tile major
    const int p0 = (wave * C::NPAIR) / C::WAVES, p1 = ((wave + 1) * C::NPAIR) / C::WAVES;
    const int nslot = p1 - p0;
    const int nt0 = p0 / C::MT;
    const int kk = lane >> 4, kap = kk & 1;
    int slot_mt[C::PPW], slot_nt[C::PPW], slot_k[C::PPW], slot_off[C::PPW];
    bool slot_neg[C::PPW], slot_row_ok[C::PPW];
#pragma unroll
    for (int s = 0; s < C::PPW; ++s) {
        const int p = p0 + (s < nslot ? s : 0);
        slot_mt[s] = p % C::MT;
        slot_nt[s] = p / C::MT;
        const int row = 16 * slot_mt[s] + (lane & 15);
        const int rho = row & 1, kw = row >> 1;
        slot_k[s] = kw / NW;
        slot_off[s] = (kw % NW) * C::WS + (rho ^ kap) - kap + kk;
        // real embedding [[Dr, -Di], [Di, Dr]]: the (re row, im column) entry is negated
        slot_neg[s] = (rho == 0 && kap == 1);
        // rows past 2*Nkz*Nw are padding: zero operand
        slot_row_ok[s] = row < C::MROWS;
        if (row >= C::MROWS) slot_k[s] = 0;
    }
    f64x4 acc[C::PPW];
#pragma unroll
    for (int s = 0; s < C::PPW; ++s) acc[s] = f64x4{0.0, 0.0, 0.0, 0.0};

    auto mfma_chunk = [&](int64_t g) {
        const int ch = (int)(g % C::NCHUNK), kp = ch / C::NP, np = ch % C::NP;
        const double* P = sP + (g & 1) * (C::KR * C::NCP);
        int abase[C::PPW];
#pragma unroll
        for (int s = 0; s < C::PPW; ++s) {
            const int q = (slot_k[s] - kp + NKZ) % NKZ;
            abase[s] = q * C::QS + np * 36 + slot_off[s];
        }
        const bool last_pair_short = (NB & 1) && (np == C::NP - 1);
#pragma unroll
        for (int ks = 0; ks < C::KS; ++ks) {
            const int kr = 4 * ks + kk;
            // the second neighbour of the last pair is padding when NB is odd
            const bool k_ok = !(last_pair_short && kr >= 18);
            const double* Prow = P + kr * C::NCP + (lane & 15);
            const double b0 = Prow[16 * nt0];
            const double b1 = (nt0 + 1 < C::NT) ? Prow[16 * (nt0 + 1)] : 0.0;
#pragma unroll
            for (int s = 0; s < C::PPW; ++s) {
                if (s < nslot) {
                    const bool ok = k_ok && slot_row_ok[s];
                    const double dv = sD[ok ? abase[s] + 4 * ks : 0];
                    const double av = ok ? (slot_neg[s] ? -dv : dv) : 0.0;
                    const double bv = (slot_nt[s] == nt0) ? b0 : b1;
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[s], 0, 0, 0);
                }
            }
        }
    };

    // ---- add this wave's V tiles of energy block blk into the output ring
    auto scatter = [&](int64_t blk) {
#pragma unroll
        for (int s = 0; s < C::PPW; ++s) {
            if (s < nslot) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * slot_mt[s] + 4 * v + (lane >> 4);
                    const int col = 16 * slot_nt[s] + (lane & 15);
                    if (row < C::MROWS && col < C::NCOLS) {
                        const int rho = row & 1, kw = row >> 1, k = kw / NW, w = kw % NW + 1;
                        const int el = col / NORB, c = col % NORB;
                        const int64_t es = blk * EB + el;
                        const double val = acc[s][v];
                        if (es < NE) {
                            const int64_t lo = es - w, hi = es + w;
                            if (lo >= 0) atomicAdd(&sR[(int)(lo % C::RING) * C::RP + (k * NORB + c) * 2 + rho], val);
                            if (hi < NE) atomicAdd(&sR[(int)(hi % C::RING) * C::RP + (k * NORB + c) * 2 + rho], val);
                        }
                    }
                }
                acc[s] = f64x4{0.0, 0.0, 0.0, 0.0};
            }
        }
    };

    // ---- scale by alpha and store output planes [e_lo, e_hi); clear their ring slots
    auto write_planes = [&](int64_t e_lo, int64_t e_hi) {
        if (e_lo < 0) e_lo = 0;
        if (e_hi > NE) e_hi = NE;
        const int per = NKZ * NORB;
        for (int64_t x = tid; x < (e_hi - e_lo) * per; x += C::THREADS) {
            const int64_t e = e_lo + x / per;
            const int kc = (int)(x % per), k = kc / NORB, c = kc % NORB;
            double* slot = sR + (int)(e % C::RING) * C::RP + kc * 2;
            const cd v{slot[0], slot[1]};
            slot[0] = 0.0;
            slot[1] = 0.0;
            cstore(S, off_S(d, k, e, a) + r * NORB + c, cmul(alpha, v));
        }
    };

    __syncthreads();
    produce_x(0);
    __syncthreads();
    produce_p(0);
    produce_x(1);
    __syncthreads();

    const bool mfma_first = wave < 4;  // waves w and w+4 share a SIMD
    for (int64_t g = 0; g < niter; ++g) {
        const bool block_end = (g % C::NCHUNK) == C::NCHUNK - 1;
        const int64_t blk = g / C::NCHUNK;
        if (mfma_first) {
            mfma_chunk(g);
        } else {
            produce_p(g + 1);
            produce_x(g + 2);
            mfma_chunk(g);
        }
        if (block_end) {
            // fixed wave order keeps the fp64 sums bitwise reproducible
            for (int w = 0; w < C::WAVES; ++w) {
                if (wave == w) scatter(blk);
                __syncthreads();
            }
            write_planes(blk * EB - NW, (blk + 1) * EB - NW);
        }
        if (mfma_first) {
            produce_p(g + 1);
            produce_x(g + 2);
        }
        __syncthreads();
    }
    write_planes(nblk * EB - NW, NE);
}

template <int NORB, int NKZ, int NW, int NB, int EB>
static hipError_t launch_fwd64(const Dims& d, const double* G, const double* D, const double* A, const int32_t* nbr,
                               cd alpha, double* S, hipStream_t stream) {
    using C = Fwd64<NORB, NKZ, NW, NB, EB>;
    auto kern = fwd_mfma64_kernel<NORB, NKZ, NW, NB, EB>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)C::LDS_BYTES);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t groups = ((d.na + 7) / 8) * 8 * NORB;
    hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(C::THREADS), C::LDS_BYTES, stream, d, G, D, A, nbr, alpha, S);
    return hipGetLastError();
}

bool fwd64_specialised(const Dims& d) {
    return (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 4) || (d.norb == 4 && d.nkz == 3 && d.nw == 2 && d.nb == 4) ||
           (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 3);
}

hipError_t launch_fwd_mfma64(const Dims& d, const double* G, const double* D, const double* A, const int32_t* nbr,
                             cd alpha, double* S, hipStream_t stream) {
    if (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 4)
        return launch_fwd64<10, 7, 10, 4, 8>(d, G, D, A, nbr, alpha, S, stream);
    if (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 3)
        return launch_fwd64<10, 7, 10, 3, 8>(d, G, D, A, nbr, alpha, S, stream);
    if (d.norb == 4 && d.nkz == 3 && d.nw == 2 && d.nb == 4)
        return launch_fwd64<4, 3, 2, 4, 8>(d, G, D, A, nbr, alpha, S, stream);
    return hipErrorInvalidValue;
}

}  // namespace sse
