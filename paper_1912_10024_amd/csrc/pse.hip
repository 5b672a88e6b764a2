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
// pse_mfma_kernel (Norb 10, Nkz 7, Nw 10, NB 4 or 3): one workgroup of 8 + NB
// waves per atom a sweeps the source points (E outer, k inner).  Per source point:
//   1. V[n][j] = A_j . Go[k, E, nbr[a,n]]          (fp64 VALU, LDS)
//   2. T[n][i][j] = V[n][j] . A_i^H                 (fp64 VALU, into two LDS planes)
//      Steps 1-2 run on four formation waves (one per neighbour slot n) one
//      source point ahead of step 3, into the other of two T buffers.
//   3. C[(q,w), (n,i,j,re/im)] += sum over (s,t,re/im) of
//        Gs[(k+q) mod Nkz, E+w, a][s][t] (re or im) * B[(s,t,re/im), (n,i,j,re/im)]
//      on the fp64 matrix cores: M = Nkz Nw = 70 rows (5 tiles), N = 2 * 9 NB = 72
//      columns (5 tiles; 54 and 4 for NB 3), K = 2 Norb^2 = 200 (50 k-steps).  B is the real
//      embedding [[Tr, Ti], [-Ti, Tr]] of T; the A rows are read straight from Gs
//      in global memory (one row = one Gs block, reused by the column tiles).
//      Eight matrix-core waves form 4 K groups (k-steps dealt round-robin) x 2
//      tile groups (13 and 12 of the 25 tiles; 10 and 10 of 20 for NB 3).
// Each SIMD runs two matrix-core waves and one formation wave, so one wave's
// load, LDS and barrier waits are covered by another's work; there is one
// barrier per source point.  After the sweep the K groups' accumulators are
// added in a fixed order in LDS, scaled by beta and written out; every output
// entry is written once.
//
// pse_generic_kernel (any other shape): one workgroup per neighbour slot, the
// same three steps on the vector ALUs with one thread per (q, w).
#include "sse_kernels.h"

namespace sse {

typedef double pse_f64x4 __attribute__((ext_vector_type(4)));

// A zero Gs block: read by the padding rows of the GEMM and by rows whose
// energy E + w leaves the grid, so the row loads need no branch.  It is never
// written; it is not declared const so that it shares the global address space
// with the input tensors and the selected pointer stays a global one (a flat
// load would also count against the LDS wait counter).
__device__ double pse_zero_block[256] = {};

template <int N, int NK, int NW, int NB>
struct PseCfg {
    static constexpr int KG = 4;                       // K groups: k-steps kg, kg + KG, ...
    static constexpr int TG = 2;                       // tile groups
    static constexpr int MWAVES = KG * TG;             // matrix-core waves
    static constexpr int FWAVES = NB;                  // formation waves, one per neighbour slot
    static constexpr int WAVES = MWAVES + FWAVES, THREADS = 64 * WAVES;
    static constexpr int NN = N * N;
    static constexpr int NCOLC = 9 * NB;               // complex GEMM columns (n, i, j)
    static constexpr int NT = (2 * NCOLC + 15) / 16;   // column tiles
    // T plane row stride (complex columns): odd, so the nine stores of a formation
    // lane (consecutive rows across lanes) hit distinct LDS banks; the padding
    // columns 2*NCOLC.. of the last tile read the next row and land in discarded outputs
    static constexpr int CPAD = NCOLC | 1;
    static constexpr int MROWS = NK * NW;              // (q, w) rows
    static constexpr int MT = (MROWS + 15) / 16;       // row tiles
    static constexpr int NTILES = MT * NT;
    static constexpr int SL = (NTILES + 1) / 2;        // tiles (accumulator slots) of tile group 0
    static constexpr int ML = (SL + NT - 1) / NT;      // row tiles a wave touches
    static constexpr int KSTEPS = NN / 2;              // 2 Norb^2 real K rows, 4 per k-step
    static constexpr int KS_MAX = (KSTEPS + KG - 1) / KG;
    // the im plane starts at an offset of 16 LDS banks (mod 32) from the re plane,
    // so a 16-lane group reading 8 columns of each plane is conflict-free
    static constexpr int PLANE = ((NN - 1) * CPAD + 8 * NT - 8) / 16 * 16 + 24;
    static constexpr int TBUF = 2 * PLANE;             // one T buffer (re, im planes), doubles
    static constexpr int VROW = N + 1;                 // padded row of a V block (complex)
    static constexpr int L_A = NB * 3 * NN * 2;        // grad H of the atom (doubles)
    static constexpr int L_V = NB * 3 * N * VROW * 2;  // V = A_j Go of each formation wave (Go before it)
    static constexpr int L_T = 2 * TBUF;               // T, double-buffered
    static constexpr int L_RED = KG * NT * 256;        // reduction scratch, aliases the T buffers
    static constexpr int L_TR = L_T > L_RED ? L_T : L_RED;
    static constexpr size_t LDS_BYTES = sizeof(double) * (L_A + L_V + L_TR);
    static constexpr int GO_PER_LANE = (NN + 63) / 64;
    static_assert(NN % 2 == 0, "K = 2 Norb^2 must split into k-steps of 4");
    static_assert(2 * NN <= 256, "zero block too small");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(NTILES - SL <= SL && ML <= MT, "tile groups");
    static_assert((NN - 1) * CPAD + 8 * NT - 1 < PLANE && PLANE % 16 == 8, "plane layout");
    static_assert(NN * 2 <= 3 * N * VROW * 2, "the Go block fits in the V block it precedes");
    static_assert(N % 2 == 0 && N * (N / 2) <= 64, "formation lanes: (t, pair of r or s) per lane");
};

// Tile of accumulator slot s: group 0 holds tiles 0 .. SL-1 in row-major
// order, group 1 the rest counted from the last tile backwards, so both
// groups run the same slot schedule with mirrored tile indices.
template <class C>
__device__ __forceinline__ int pse_tile_mt(int tg, int s) { return tg ? C::MT - 1 - s / C::NT : s / C::NT; }
template <class C>
__device__ __forceinline__ int pse_tile_nt(int tg, int s) { return tg ? C::NT - 1 - s % C::NT : s % C::NT; }

// Sum of the K groups' partial results of row tile mt (in K-group order), scaled
// by beta and written to Pi; run by every thread of the workgroup.
template <class C, int NW>
__device__ __forceinline__ void pse_sum_row_tile(const Dims& d, const double* red, int mt, int tid, int64_t a, cd beta,
                                                 double* __restrict__ Pi) {
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
}

// MODE = 0: Pi (Eq. 4) with Gs, Go as documented above.
// MODE != 0: the D part of the adjoint of Eq. 3 for dL/dSigma = g,
//   dD[q, w-1, a, n][i][j] = conj(alpha) sum_{k', E'} sum_{s in S} [0 <= E' + s w < NE]
//                            sum_{r,c} conj((A_i G[k', E', b] A_j^H)[r][c]) g[k'+q, E'+s w, a][r][c],
// which is the same contraction with Gs := g (no slot axis), the energy
// branches of S summed into each A row, and T_ij = A_j . G^H . A_i^H (the Go
// block is staged conjugate-transposed); beta = conj(alpha).  MODE is the set
// S: bit 0 the branch s = +1 (g at E' + w: the terms whose G sits at E - w,
// i.e. the coefficients at +w), bit 1 the branch s = -1 (coefficients at -w);
// the one-table form of Eq. 3 takes both.
// AM (adjoint only): g is read from its atom-major copy (pse_atom_major_g):
// the GEMM rows of one workgroup then come from one contiguous region of the
// atom (a few pages) instead of one (k, E) slab per block, 147 of them for the
// 21 energies x 7 momenta a workgroup reads at a time.  Same arithmetic in the
// same order as AM = false.
template <int N, int NK, int NW, int NB, int MODE, bool AM>
__global__ __launch_bounds__(64 * (8 + NB)) void pse_mfma_kernel(
    Dims d, const double* __restrict__ Gs, const double* __restrict__ Go, const double* __restrict__ Ag,
    const int32_t* __restrict__ nbr, cd beta, double* __restrict__ Pi) {
    using C = PseCfg<N, NK, NW, NB>;
    static_assert(C::THREADS == 64 * (8 + NB), "launch bounds");
    constexpr bool ADJ = MODE != 0, UP = !ADJ || (MODE & 1) != 0, LO = ADJ && (MODE & 2) != 0;
    static_assert(!AM || ADJ, "the atom-major copy is the adjoint's");
    constexpr int NN = C::NN;
    extern __shared__ __align__(16) double smem[];
    double* sA = smem;           // [NB][3][N][N] complex
    double* sV = sA + C::L_A;    // [NB][3 (j)][N (t)][VROW (r)] complex, per formation wave; the
                                 // wave's Go block [N][N] sits at its start until V is written
    double* sT = sV + C::L_V;    // two buffers; each: re plane [NN][CPAD], im plane at +PLANE;
                                 // entry (s*N + t, n*9 + i*3 + j) = T_ij[t][s]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t a = blockIdx.x;
    const int NE = (int)d.ne;
    const int64_t NA = d.na;
    const int64_t slot = 2 * d.gs * NN;   // doubles between atoms at one (k, E)
    const int64_t e_step = slot * NA;      // doubles between energies
    const int64_t k_step = e_step * NE;    // doubles between momenta
    // the shifted operand: Gs (laid out like G) or, for the adjoint, g (one block per
    // atom), in its own layout or atom-major ([a][k][E] blocks)
    const int64_t rs_slot = ADJ ? (AM ? 2 * NN * NE * (int64_t)NK : 2 * NN) : slot;
    const int64_t rs_e = AM ? 2 * NN : rs_slot * NA, rs_k = AM ? 2 * NN * (int64_t)NE : rs_e * NE;
    const int nsrc = NK * NE;

    for (int x = tid; x < NB * 3 * NN; x += C::THREADS) {
        const cd v = cload(Ag, off_A(d, a, 0, 0) + x);
        sA[2 * x] = v.re;
        sA[2 * x + 1] = v.im;
    }
    for (int x = tid; x < C::L_TR; x += C::THREADS) sT[x] = 0.0;
    __syncthreads();

    if (wave >= C::MWAVES) {
        // ---------------- formation wave of neighbour slot n: T[n] of every source point
        const int n = wave - C::MWAVES;
        // T of the next source point must be ready by the barrier that ends the
        // matrix-core waves' current one: the formation wave's instructions go first
        __builtin_amdgcn_s_setprio(2);
        const int32_t b = nbr[a * NB + n];
        const bool b_ok = b >= 0 && b < NA;
        const int64_t go_base = b_ok ? slot * b : 0;
        double* myV = sV + n * 3 * N * C::VROW * 2;
        double* myGo = myV;
        const double* myA = sA + n * 3 * NN * 2;
        cd gv[C::GO_PER_LANE];
        auto load_go = [&](int src) {
            const int E = src / NK, k = src % NK;
            const double* blk = b_ok ? Go + k * k_step + (int64_t)E * e_step + go_base : pse_zero_block;
#pragma unroll
            for (int u = 0; u < C::GO_PER_LANE; ++u) {
                const int x = lane + 64 * u;
                const double2 v = *reinterpret_cast<const double2*>(blk + 2 * (x < NN ? x : 0));
                gv[u] = cd{v.x, v.y};
            }
        };
        auto form = [&](int src, double* T) {
#pragma unroll
            for (int u = 0; u < C::GO_PER_LANE; ++u) {
                const int x = lane + 64 * u;
                if (x < NN) {
                    if constexpr (ADJ)   // G^H: element (r, c) of G goes to (c, r), conjugated
                        *reinterpret_cast<double2*>(myGo + 2 * ((x % N) * N + x / N)) = make_double2(gv[u].re, -gv[u].im);
                    else
                        *reinterpret_cast<double2*>(myGo + 2 * x) = make_double2(gv[u].re, gv[u].im);
                }
            }
            if (src + 1 < nsrc) load_go(src + 1);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // V[j][t][r] = sum_u A[j][t][u] Go[u][r]; a lane owns (t, r0 = rp, r1 = rp + N/2)
            // for the three j, kept in registers until every lane has read Go
            constexpr int RH = N / 2;
            const bool f_lane = lane < N * RH;
            const int ft = f_lane ? lane / RH : 0, fp = lane % RH;
            cd vres[2][3];
            {
                const double* A0 = myA + 2 * ft * N;
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int j = 0; j < 3; ++j) vres[h][j] = cd{0.0, 0.0};
#pragma unroll 2
                for (int u = 0; u < N; ++u) {
                    const cd g0{myGo[2 * (u * N + fp)], myGo[2 * (u * N + fp) + 1]};
                    const cd g1{myGo[2 * (u * N + fp + RH)], myGo[2 * (u * N + fp + RH) + 1]};
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const cd av{A0[2 * (j * NN + u)], A0[2 * (j * NN + u) + 1]};
                        cfma(vres[0][j], av, g0);
                        cfma(vres[1][j], av, g1);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (f_lane) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    double* V0 = myV + 2 * (ft * C::VROW + fp + h * RH);
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        *reinterpret_cast<double2*>(V0 + 2 * j * N * C::VROW) = make_double2(vres[h][j].re, vres[h][j].im);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // T[i][j][t][s] = sum_r V[j][t][r] conj(A[i][s][r]); a lane owns (t, s0 = sp, s1 = sp + N/2),
            // rows kap = s*N + t of the T planes (consecutive lanes, consecutive rows)
            if (f_lane) {
                const int t = lane % N, sp = lane / N;
                const double* V0 = myV + 2 * t * C::VROW;
                const double* A0 = myA + 2 * sp * N;
                cd tv[2][9];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int ij = 0; ij < 9; ++ij) tv[h][ij] = cd{0.0, 0.0};
#pragma unroll 2
                for (int r = 0; r < N; ++r) {
                    cd vj[3];
#pragma unroll
                    for (int m = 0; m < 3; ++m) vj[m] = cd{V0[2 * (m * N * C::VROW + r)], V0[2 * (m * N * C::VROW + r) + 1]};
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            const double* Ai = A0 + 2 * (i * NN + h * RH * N + r);
                            const cd ai{Ai[0], Ai[1]};
#pragma unroll
                            for (int j = 0; j < 3; ++j) cfma_conj(tv[h][i * 3 + j], vj[j], ai);
                        }
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    double* T0 = T + ((sp + h * RH) * N + t) * C::CPAD + n * 9;
#pragma unroll
                    for (int ij = 0; ij < 9; ++ij) {
                        T0[ij] = tv[h][ij].re;
                        T0[C::PLANE + ij] = tv[h][ij].im;
                    }
                }
            }
        };
        load_go(0);
        form(0, sT);
        __syncthreads();
        for (int src = 0; src < nsrc; ++src) {
            if (src + 1 < nsrc) form(src + 1, sT + ((src + 1) & 1) * C::TBUF);
            __syncthreads();
        }
        // the same barrier sequence as the matrix-core waves' reduction
        for (int mt = 0; mt < C::MT; ++mt) {
            if (mt > 0) __syncthreads();
            __syncthreads();
            pse_sum_row_tile<C, NW>(d, sT, mt, tid, a, beta, Pi);
        }
    } else {
        // ---------------- matrix-core wave: K group kg, tile group tg
        // waves w and w + KG share a SIMD; pairing tile group 0 of K group g with tile
        // group 1 of K group g + KG/2 evens out the matrix-core work per SIMD (the
        // K groups own 13 or 12 k-steps, the tile groups 13 or 12 tiles)
        const int tg = wave / C::KG, kg = (wave % C::KG + tg * (C::KG / 2)) % C::KG;
        // A (16 x 4 per k-step): lane holds row j16, K index kk; B (4 x 16): K index kk,
        // column j16.  K index 4 ks + kk = (Gs element s*N + t = 2 ks + kk/2, re/im = kk & 1).
        const int kk = lane >> 4, j16 = lane & 15, kc = kk & 1;
        // B: plane (re or im) and sign of this lane's entry of [[Tr, Ti], [-Ti, Tr]]
        int boff[C::NT];
        int b_neg;   // sign bit of the high word
        {
            const int dd = j16 & 1;
            const int plane = (kc ^ dd) ? C::PLANE : 0;
            b_neg = (kc == 1 && dd == 0) ? (int)0x80000000u : 0;
#pragma unroll
            for (int nl = 0; nl < C::NT; ++nl) {
                const int nt = tg ? C::NT - 1 - nl : nl;
                boff[nl] = plane + (kk >> 1) * C::CPAD + 8 * nt + (j16 >> 1) + 2 * kg * C::CPAD;
            }
        }
        const bool last_slot = tg == 0;   // group 0 owns one tile more when NTILES is odd

        pse_f64x4 acc[C::SL];
#pragma unroll
        for (int s = 0; s < C::SL; ++s) acc[s] = pse_f64x4{0.0, 0.0, 0.0, 0.0};

        // A rows of a source point: the wave's first k-step and the lane's K index folded
        // in; the adjoint adds the row of the lower energy branch (ap2)
        const double* ap[C::ML];
        const double* ap2[C::ML];
        auto a_rows = [&](int src) {
            const int E = src / NK, k = src % NK;
#pragma unroll
            for (int ml = 0; ml < C::ML; ++ml) {
                const int r = 16 * (tg ? C::MT - 1 - ml : ml) + j16;   // GEMM row (q, w)
                const int w = r % NW + 1, es = E + w;
                const bool ok = r < C::MROWS && es < NE;
                const int kq = (k + r / NW) % NK;
                const double* base = Gs + kq * rs_k + rs_slot * a;
                ap[ml] = (ok ? base + (int64_t)es * rs_e : pse_zero_block) + 4 * kg + kk;
                if constexpr (LO) {
                    const bool ok2 = r < C::MROWS && E - w >= 0;
                    ap2[ml] = (ok2 ? base + (int64_t)(E - w) * rs_e : pse_zero_block) + 4 * kg + kk;
                }
            }
        };
        auto a_load = [&](int ml, int off) {
            if constexpr (UP && LO)
                return ap[ml][off] + ap2[ml][off];
            else if constexpr (LO)
                return ap2[ml][off];
            else
                return ap[ml][off];
        };
        double an[C::ML];
        a_rows(0);
#pragma unroll
        for (int ml = 0; ml < C::ML; ++ml) an[ml] = a_load(ml, 0);
        __syncthreads();   // T of source point 0 is formed
        for (int src = 0; src < nsrc; ++src) {
            const double* Tb = sT + (src & 1) * C::TBUF;
#pragma unroll
            for (int i = 0; i < C::KS_MAX; ++i) {
                const bool live = kg + C::KG * i < C::KSTEPS;
                double ac[C::ML];
#pragma unroll
                for (int ml = 0; ml < C::ML; ++ml) ac[ml] = an[ml];
                if (i + 1 < C::KS_MAX && kg + C::KG * (i + 1) < C::KSTEPS) {
#pragma unroll
                    for (int ml = 0; ml < C::ML; ++ml) an[ml] = a_load(ml, 4 * C::KG * (i + 1));
                } else if (src + 1 < nsrc) {
                    // last k-step of this source point: the next point's first rows
                    a_rows(src + 1);
#pragma unroll
                    for (int ml = 0; ml < C::ML; ++ml) an[ml] = a_load(ml, 0);
                }
                if (live) {
                    double bv[C::NT];
#pragma unroll
                    for (int nl = 0; nl < C::NT; ++nl)
                    {
                        const double x = Tb[boff[nl] + 2 * C::KG * i * C::CPAD];
                        bv[nl] = __hiloint2double(__double2hiint(x) ^ b_neg, __double2loint(x));
                    }
#pragma unroll
                    for (int s = 0; s < C::SL; ++s) {
                        if (s == C::SL - 1 && C::SL * 2 != C::NTILES && !last_slot) continue;
                        acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[s / C::NT], bv[s % C::NT], acc[s], 0, 0, 0);
                    }
                }
            }
            __syncthreads();   // the next T buffer is formed; this one may be overwritten
        }
        // partial sums of the K groups, one row tile at a time
        double* red = sT;   // [KG][NT][16 rows][16 cols]
        for (int mt = 0; mt < C::MT; ++mt) {
            if (mt > 0) __syncthreads();   // the previous row tile is read
#pragma unroll
            for (int s = 0; s < C::SL; ++s) {
                if (s == C::SL - 1 && C::SL * 2 != C::NTILES && !last_slot) continue;
                if (pse_tile_mt<C>(tg, s) != mt) continue;
                const int nt = pse_tile_nt<C>(tg, s);
#pragma unroll
                for (int v = 0; v < 4; ++v) red[(kg * C::NT + nt) * 256 + (4 * v + (lane >> 4)) * 16 + j16] = acc[s][v];
            }
            __syncthreads();
            pse_sum_row_tile<C, NW>(d, red, mt, tid, a, beta, Pi);
        }
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
    return d.norb == 10 && d.nkz == 7 && d.nqz == 7 && d.nw == 10 && (d.nb == 4 || d.nb == 3) && d.ne < (1 << 28);
}

template <int NB, int MODE, bool AM = false>
static hipError_t launch_pse_mfma(const Dims& d, const double* Rs, const double* Go, const double* A,
                                  const int32_t* nbr, cd beta, double* out, hipStream_t stream) {
    using C = PseCfg<10, 7, 10, NB>;
    auto kern = pse_mfma_kernel<10, 7, 10, NB, MODE, AM>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)C::LDS_BYTES);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)d.na), dim3(C::THREADS), C::LDS_BYTES, stream, d, Rs, Go, A, nbr, beta, out);
    return hipGetLastError();
}

bool pse_generic_supported(const Dims& d) {
    return d.nqz * d.nw <= 2 * kPseThreads && pse_generic_lds(d) <= 160 * 1024 && d.na * d.nb <= INT32_MAX;
}

hipError_t launch_pse(const Dims& d, const double* Gs, const double* Go, const double* A, const int32_t* nbr, cd beta,
                      double* Pi, hipStream_t stream) {
    if (pse_mfma_specialised(d))
        return d.nb == 4 ? launch_pse_mfma<4, 0, false>(d, Gs, Go, A, nbr, beta, Pi, stream)
                         : launch_pse_mfma<3, 0, false>(d, Gs, Go, A, nbr, beta, Pi, stream);
    const size_t lds = pse_generic_lds(d);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(pse_generic_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pse_generic_kernel, dim3((unsigned)(d.na * d.nb)), dim3(kPseThreads), lds, stream, d, Gs, Go, A,
                       nbr, beta, Pi);
    return hipGetLastError();
}

template <int MODE, bool AM>
static hipError_t launch_dd_mode(const Dims& d, const double* G, const double* A, const int32_t* nbr, const double* gS,
                                 cd calpha, double* dD, hipStream_t stream) {
    return d.nb == 4 ? launch_pse_mfma<4, MODE, AM>(d, gS, G, A, nbr, calpha, dD, stream)
                     : launch_pse_mfma<3, MODE, AM>(d, gS, G, A, nbr, calpha, dD, stream);
}

template <bool AM>
static hipError_t launch_dd_layout(const Dims& d, const double* G, const double* A, const int32_t* nbr,
                                   const double* g, cd calpha, double* dD, hipStream_t stream, int branches) {
    if (branches == 3) return launch_dd_mode<3, AM>(d, G, A, nbr, g, calpha, dD, stream);
    if (branches == 1) return launch_dd_mode<1, AM>(d, G, A, nbr, g, calpha, dD, stream);
    if (branches == 2) return launch_dd_mode<2, AM>(d, G, A, nbr, g, calpha, dD, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_dd_mfma(const Dims& d, const double* G, const double* A, const int32_t* nbr, const double* gS,
                          const double* gT, cd calpha, double* dD, hipStream_t stream, int branches) {
    return gT ? launch_dd_layout<true>(d, G, A, nbr, gT, calpha, dD, stream, branches)
              : launch_dd_layout<false>(d, G, A, nbr, gS, calpha, dD, stream, branches);
}

// ------------------------------------------------------------------ atom-major copy of g
// gT[a][k][e][NN] (complex) = g[k][e][a][NN]: every entry written on every call
__global__ void pse_atom_major_kernel(int64_t nkz, int64_t ne, int64_t na, int64_t nn, const double2* __restrict__ g,
                                      double2* __restrict__ gT) {
    const int64_t per_atom = nkz * ne * nn, total = na * per_atom;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = x / per_atom, r = x % per_atom, blk = r / nn, rc = r % nn;
        gT[x] = g[(blk * na + a) * nn + rc];
    }
}

bool pse_atom_major_ok(const Dims& d) { return pse_mfma_specialised(d); }

size_t pse_atom_major_bytes(const Dims& d) {
    return pse_atom_major_ok(d) ? (size_t)(16 * d.norb * d.norb * d.nkz * d.ne * d.na + 255) / 256 * 256 : 0;
}

hipError_t pse_atom_major_g(const Dims& d, const double* g, double* gT, hipStream_t stream) {
    const int64_t n = d.na * d.nkz * d.ne * d.norb * d.norb;
    const unsigned grid = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL(pse_atom_major_kernel, dim3(grid), dim3(256), 0, stream, d.nkz, d.ne, d.na, d.norb * d.norb,
                       reinterpret_cast<const double2*>(g), reinterpret_cast<double2*>(gT));
    return hipGetLastError();
}

}  // namespace sse
