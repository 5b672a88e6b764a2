// Matrix-core forward kernel of the scattering self-energy (Eq. 3), with fp64 or
// fp32 GEMM operands (the split 16-bit forms are in fwd_h16.hip).
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
// Pipeline per chunk (one barrier): every wave gathers the G columns of a
// later chunk into registers, issues its share of the MFMAs on the P chunk in
// LDS, forms P tiles of the next chunk from the X = grad_i H . G rows in LDS
// (a second small GEMM), and forms the X rows of the chunk after that on the
// vector ALUs (double-buffered in LDS).  The two waves of a SIMD run these
// phases in opposite orders, so the latency-bound phases of one wave meet
// the matrix work of the other.  The host launches the atoms in batches of
// about twelve rounds of workgroups, so that the row workgroups of an atom
// keep sharing its neighbours' G blocks in L2.  At the end of an energy block the waves add
// their accumulators into a ring of output planes (LDS, fp64) in phases that
// touch disjoint entries, so results are bitwise reproducible; planes that
// can receive no more contributions are scaled by alpha and written out.
#include <algorithm>
#include <type_traits>

#include "fwd_common.h"
#include "sse_kernels.h"

namespace sse {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Operand type of the matrix-core GEMM: fp64 (16x16x4 f64 MFMA) or fp32
// (16x16x4 f32 MFMA, fp32 accumulation over one K chunk, then fp64).
template <int PREC>
struct Oper;
template <>
struct Oper<SSE_FP64> {
    using T = double;
    using Acc = f64x4;
    static __device__ __forceinline__ Acc mma(T a, T b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ T neg_if(T x, bool neg) {
        return __longlong_as_double(__double_as_longlong(x) ^ (neg ? (long long)0x8000000000000000ull : 0ll));
    }
    // C[i][j] of a 16x16 tile sits in lane j + 16*(i%4), register i/4
    static __device__ __forceinline__ int row_of(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <>
struct Oper<SSE_FP32> {
    using T = float;
    using Acc = f32x4;
    static __device__ __forceinline__ Acc mma(T a, T b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ T neg_if(T x, bool neg) {
        return __int_as_float(__float_as_int(x) ^ (neg ? (int)0x80000000u : 0));
    }
    // C[i][j] of a 16x16 tile sits in lane j + 16*(i/4), register i%4
    static __device__ __forceinline__ int row_of(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// HBA: the right factor of Eq. 3 is a stored grad_j H_ba (its own table in LDS
// for the P tiles) instead of grad_j H^H
template <int NORB, int NKZ, int NW, int NB, int EB, int PREC, bool HBA>
struct Fwd64 {
    using T = typename Oper<PREC>::T;
    static constexpr int WAVES = 8, THREADS = 64 * WAVES;
    static constexpr int MROWS = 2 * NKZ * NW;
    static constexpr int MT = (MROWS + 15) / 16;
    static constexpr int NCOLS = EB * NORB;
    static constexpr int NT = (NCOLS + 15) / 16;
    static constexpr int NCP = NT * 16;
    static constexpr int NP = (NB + 1) / 2;      // neighbour pairs per k'
    static constexpr int NB2 = 2 * NP;           // neighbour slots in the D table (odd NB padded)
    static constexpr int NCHUNK = NKZ * NP;
    static constexpr int KR = 36;
    static constexpr int KS = 9;
    static constexpr int RING = EB + 2 * NW;
    static constexpr int WS = NB2 * 18 + 2;      // D-table stride per w, padded to spread LDS banks
    static constexpr int QS = NW * WS;
    static constexpr int ZOFF = NKZ * QS;        // zero region read by padding rows
    static constexpr int NN = NORB * NORB;
    static constexpr int NWV = NW;
    // wave -> M-tile ownership: waves own whole M-tiles (all N-tiles); the
    // M-tiles past the eighth are dealt out one (M-tile, N-tile) pair per wave
    static constexpr int OWN = MT < WAVES ? MT : WAVES;
    static constexpr int XP = MT > WAVES ? (MT - WAVES) * NT : 0;
    // LDS carve-up: D table and P chunks in the operand type, the rest in doubles
    static constexpr int L_D = ZOFF + NP * 36 + 4;
    // grad H in LDS: one block per neighbour pair ([nl][i][r][t] complex, a padding
    // slot of an odd Nb stays zero), each followed by a zero tail that padding
    // lanes of the P tiles read.  Rows (r) are padded to an odd number of
    // doubles so that the 16 lanes of a P-tile operand load, which read 16
    // consecutive (j, c) rows, hit distinct LDS banks.
    static constexpr int AR = 2 * NORB + 1;       // doubles per grad H row
    static constexpr int NNS = NORB * AR;         // doubles per grad H block
    static constexpr int ZT = 2 * NORB + 2;
    static constexpr int PSTR = 2 * 3 * NNS + ZT;
    static constexpr int L_A = NP * PSTR;
    // two P buffers; the slot after each takes the padding results of the P tiles
    static constexpr int PBS = KR * NCP + 2;
    static constexpr int TRASH = KR * NCP;
    static constexpr int L_P = 2 * PBS;
    // one X buffer: rows [nl][el][i] of Norb complex, padded to XR doubles so that
    // the rows a P tile reads (consecutive (el, i) of one nl) spread over the
    // LDS banks, and kept even so a (re, im) pair is one 16-byte store
    static constexpr int XR = 2 * NORB + 2;
    static constexpr int XB = 2 * EB * 3 * XR;
    // P tiles run on fp64 MFMAs for the fp64 form and on fp32 MFMAs otherwise;
    // their operands (X rows and a copy of the right factor) are stored in that
    // type; the fp64 form shares the grad H table with the X rows unless the
    // right factor is a stored grad H_ba
    using TPT = typename Oper<PREC == SSE_FP64 ? SSE_FP64 : SSE_FP32>::T;
    static constexpr bool SPLIT_A = PREC != SSE_FP64 || HBA;
    static constexpr int L_X = (2 * XB * (int)sizeof(TPT) + 7) / 8;
    static constexpr int L_AP = SPLIT_A ? (L_A * (int)sizeof(TPT) + 7) / 8 : 0;
    static constexpr int RP = NKZ * NORB * 2;  // one ring plane: [k][c] complex
    static constexpr int L_R = RING * RP;
    static constexpr int OPER_DOUBLES = ((L_D + L_P) * (int)sizeof(T) + 7) / 8;
    static constexpr size_t LDS_BYTES = sizeof(double) * (size_t)(OPER_DOUBLES + L_A + L_AP + L_X + L_R);
    static constexpr int X_ITEMS = EB * 2 * 3 * NORB;  // (el, nl, i, u)
    static constexpr int X_IPW = (X_ITEMS + WAVES - 1) / WAVES;
    // P chunk on the matrix cores, per neighbour of the pair: C[(el,i,re/im), (j,c)] =
    // sum_(u,re/im) X-embedding[(el,i,re/im), (u,re/im)] . conj(gradH[n][j][c][u]) parts
    static constexpr int PM_ROWS = EB * 3 * 2;
    static constexpr int PMT = (PM_ROWS + 15) / 16;
    static constexpr int PKS = (2 * NORB + 3) / 4;
    static constexpr int PNC = 3 * NORB;
    static constexpr int PNT = (PNC + 15) / 16;
    static constexpr int NPT = 2 * PMT * PNT;     // P tiles per chunk
    // issue cost of one P tile in main-GEMM k-steps (fp64 and fp32 alike)
    static constexpr int PTILE_COST = PKS;
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(X_IPW <= 64, "one item per lane");
    static_assert(NPT <= 32, "P tiles fit a 32-bit wave mask");
    static_assert(XP <= WAVES, "at most one extra (M-tile, N-tile) pair per wave");
    static_assert(NKZ <= 32, "momentum sets of a tile fit a 32-bit mask");
};

// Static deal of the P tiles of a chunk to waves: each tile goes to a wave on
// the SIMD with the least issue time so far (the two waves of SIMD s are s
// and s + 4), ties to the wave with fewer tiles.
template <class C>
struct PTileDeal {
    uint32_t mask[C::WAVES];
    int count[C::WAVES];
    int maxper;
    constexpr PTileDeal() : mask{}, count{}, maxper(0) {
        int simd_load[4] = {0, 0, 0, 0};
        for (int w = 0; w < C::WAVES; ++w)
            simd_load[w % 4] += (w < C::OWN ? C::NT * C::KS : 0) + (w < C::XP ? C::KS : 0);
        for (int t = 0; t < C::NPT; ++t) {
            int best = 0;
            for (int w = 1; w < C::WAVES; ++w) {
                const int lw = simd_load[w % 4], lb = simd_load[best % 4];
                if (lw < lb || (lw == lb && count[w] < count[best])) best = w;
            }
            simd_load[best % 4] += C::PTILE_COST;
            mask[best] |= 1u << t;
            ++count[best];
        }
        for (int w = 0; w < C::WAVES; ++w)
            if (count[w] > maxper) maxper = count[w];
    }
};

template <int NORB, int NKZ, int NW, int NB, int EB, int PREC, int FLAGS, bool HBA>
__global__ __launch_bounds__(512) void fwd_mfma_kernel(Dims d, const double* __restrict__ G,
                                                       const double* __restrict__ Dg,
                                                       const double* __restrict__ Ag,
                                                       const double* __restrict__ Bg,
                                                       const int32_t* __restrict__ nbr, cd alpha,
                                                       double* __restrict__ S, int64_t a0) {
    using C = Fwd64<NORB, NKZ, NW, NB, EB, PREC, HBA>;
    using O = Oper<PREC>;
    using T = typename O::T;
    constexpr PTileDeal<C> deal{};
    constexpr int MAXT = deal.maxper;
    extern __shared__ double lds[];
    T* sD = reinterpret_cast<T*>(lds);
    T* sP = sD + C::L_D;
    // P chunks are formed on the fp64 matrix cores for the fp64 form, on the fp32
    // ones otherwise
    using OP = Oper<PREC == SSE_FP64 ? SSE_FP64 : SSE_FP32>;
    using TP = typename OP::T;
    double* sA = lds + C::OPER_DOUBLES;
    TP* sAp = reinterpret_cast<TP*>(sA + (C::SPLIT_A ? C::L_A : 0));  // right factor for the P tiles
    TP* sX = reinterpret_cast<TP*>(sA + C::L_A + C::L_AP);
    double* sR = sA + C::L_A + C::L_AP + C::L_X;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // XCD-aware mapping: the Norb workgroups of one atom share its D, grad H and
    // neighbour G blocks, so they get block ids that land on the same XCD; this
    // launch covers the atoms from a0 (a multiple of 8).
    const int64_t bid = blockIdx.x;
    const int r = (int)((bid >> 3) % NORB);
    const int64_t a = a0 + ((bid >> 3) / NORB) * 8 + (bid & 7);
    if (a >= d.na) return;  // uniform for the whole workgroup, before any barrier

    // ---- stage the atom's D table, grad H; clear buffers
    for (int x = tid; x < C::L_D; x += C::THREADS) sD[x] = T(0);
    for (int x = tid; x < C::L_A; x += C::THREADS) sA[x] = 0.0;
    if constexpr (C::SPLIT_A)
        for (int x = tid; x < C::L_A; x += C::THREADS) sAp[x] = TP(0);
    __syncthreads();
    for (int x = tid; x < NKZ * NW * NB * 9; x += C::THREADS) {
        const int ij = x % 9, n = (x / 9) % NB, w = (x / (9 * NB)) % NW, q = x / (9 * NB * NW);
        const cd v = cload(Dg, off_D(d, q, w, a, n) + ij);
        T* o = sD + q * C::QS + w * C::WS + n * 18 + ij * 2;
        o[0] = T(v.re);
        o[1] = T(v.im);
    }
    for (int x = tid; x < NB * 3 * C::NN; x += C::THREADS) {
        const cd v = cload(Ag, off_A(d, a, 0, 0) + x);
        const int n = x / (3 * C::NN), i = (x / C::NN) % 3, rc = x % C::NN;
        const int o = (n >> 1) * C::PSTR + ((n & 1) * 3 + i) * C::NNS + (rc / NORB) * C::AR + 2 * (rc % NORB);
        sA[o] = v.re;
        sA[o + 1] = v.im;
        if constexpr (HBA) {
            // the P tiles form X . conj(table)^T: the table holds conj(B_j[u][c]) at [c][u]
            const cd b = cload(Bg, off_A(d, a, n, i) + (rc % NORB) * NORB + rc / NORB);
            sAp[o] = TP(b.re);
            sAp[o + 1] = TP(-b.im);
        } else if constexpr (C::SPLIT_A) {
            sAp[o] = TP(v.re);
            sAp[o + 1] = TP(v.im);
        }
    }
    for (int x = tid; x < C::L_P; x += C::THREADS) sP[x] = T(0);
    for (int x = tid; x < C::L_R; x += C::THREADS) sR[x] = 0.0;

    // chunk and energy indices fit 32 bits: the dispatcher admits ne < 2^28
    const int NE = (int)d.ne;
    const int nblk = (NE + EB - 1) / EB;
    const int niter = nblk * C::NCHUNK;
    const int kk = lane >> 4, kap = kk & 1, j16 = lane & 15;

    // ---- X rows, step 1: gather this lane's G column for chunk g into registers
    const int x_item = wave * C::X_IPW + lane;
    const bool x_lane = lane < C::X_IPW && x_item < C::X_ITEMS;
    const int x_u = x_item % NORB, x_i = (x_item / NORB) % 3, x_nl = (x_item / (3 * NORB)) % 2,
              x_el = x_item / (6 * NORB);
    // neighbour atom of this lane's slot in each pair: its offset into G (in
    // doubles) and whether it is valid (a padding slot or an entry outside
    // [0, na) contributes zero)
    const int64_t na = d.na, g_stride = d.gs * C::NN;
    const int64_t e_step = 2 * g_stride * na, kp_step = e_step * NE;
    int64_t b_off[C::NP];
    bool b_ok[C::NP];
#pragma unroll
    for (int p = 0; p < C::NP; ++p) {
        const int n = 2 * p + x_nl;
        const int32_t b = n < NB ? nbr[a * NB + n] : -1;
        b_ok[p] = x_lane && b >= 0 && b < na;
        b_off[p] = b_ok[p] ? 2 * g_stride * b + 2 * x_u : 0;
    }
    // Branch-free gather: an invalid lane loads from the start of G (in bounds)
    // and finish_x writes zero for it.
    cd gv[NORB];
    bool g_ok = false;
    auto gather_g = [&](int g) {
        const int gg = g < niter ? g : 0;
        const int blk = gg / C::NCHUNK;
        const int ch = gg % C::NCHUNK, kp = ch / C::NP, np = ch % C::NP;
        int64_t off = b_off[0];
        bool ok = b_ok[0];
#pragma unroll
        for (int p = 1; p < C::NP; ++p) {
            off = np == p ? b_off[p] : off;
            ok = np == p ? b_ok[p] : ok;
        }
        const int e = blk * EB + x_el;
        g_ok = g < niter && ok && e < NE;
        off += kp * kp_step + (int64_t)e * e_step;
        const double* Gb = G + (g_ok ? off : 0);
#pragma unroll
        for (int t = 0; t < NORB; ++t) gv[t] = cd{Gb[2 * t * NORB], Gb[2 * t * NORB + 1]};
    };
    // ---- X rows, step 2: X[el][nl][i][u] = sum_t gradH[n][i][r][t] G[t][u]
    auto finish_x = [&](int g) {
        if (g >= niter || !x_lane) return;
        const int np = (g % C::NCHUNK) % C::NP;
        const double* Ar = sA + np * C::PSTR + (x_nl * 3 + x_i) * C::NNS + r * C::AR;
        cd acc{0.0, 0.0};
#pragma unroll
        for (int t = 0; t < NORB; ++t) cfma(acc, cd{Ar[2 * t], Ar[2 * t + 1]}, gv[t]);
        if (!g_ok) acc = cd{0.0, 0.0};
        TP* X = sX + (g & 1) * C::XB + ((x_nl * EB + x_el) * 3 + x_i) * C::XR + 2 * x_u;
        if constexpr (PREC != SSE_FP64)  // the P tiles run on fp32 operands
            *reinterpret_cast<float2*>(X) = make_float2((float)acc.re, (float)acc.im);
        else
            *reinterpret_cast<double2*>(X) = make_double2(acc.re, acc.im);
    };

    // ---- P tiles of this wave: per-lane operand and output offsets, fixed for the
    // whole sweep (only the X/P buffer parity and the neighbour pair change)
    const uint32_t my_tiles = deal.mask[wave];
    const int my_count = deal.count[wave];
    // Real embedding of P = X . grad_j H^H with B = (Re, Im) of conj(grad H): the
    // sign of the Im part is moved onto A, whose (Im row, Im column) entry then
    // carries the only negation.  Rows past the X rows read the zero tail of the
    // first grad H block, and so do columns past the 3 Norb (j, c) columns.
    constexpr bool A_PAD = C::PM_ROWS % 16 != 0;
    constexpr int ZTAIL = 2 * 3 * C::NNS;  // offset of the zero tail inside a pair block
    int pt_a[MAXT > 0 ? MAXT : 1];        // X-embedding offset (doubles) in an X buffer
    bool pt_aok[MAXT > 0 ? MAXT : 1];     // false: the row is padding
    int pt_b[MAXT > 0 ? MAXT : 1];        // grad H offset (doubles) in a pair block
    int pt_out[MAXT > 0 ? MAXT : 1][4];   // P offsets of the four results (padding: the spare slot)
    bool pt_neg[MAXT > 0 ? MAXT : 1];
    {
        uint32_t rest = my_tiles;
#pragma unroll
        for (int si = 0; si < MAXT; ++si) {
            const int t = rest ? __builtin_ctz(rest) : 0;
            rest &= rest - 1;
            const int nt_p = t % C::PNT, mt_p = (t / C::PNT) % C::PMT, nl = t / (C::PNT * C::PMT);
            const int arow = 16 * mt_p + j16;
            const int am = arow >> 1, arho = arow & 1, ael = am / 3, ai = am % 3;
            // K index 4 ks + kk = (u = 2 ks + kk/2, re/im = kap)
            pt_aok[si] = arow < C::PM_ROWS;
            pt_a[si] = ((nl * EB + ael) * 3 + ai) * C::XR + (arho ^ kap) + 2 * (kk >> 1);
            pt_neg[si] = arho == 1 && kap == 1;
            const int bcol = 16 * nt_p + j16;
            const int bj = bcol / NORB, bc = bcol % NORB;
            pt_b[si] = (bcol < C::PNC ? (nl * 3 + bj) * C::NNS + bc * C::AR : ZTAIL) + kap + 2 * (kk >> 1);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * mt_p + OP::row_of(lane, v);
                const int m = row >> 1, rho = row & 1, el = m / 3, i = m % 3;
                pt_out[si][v] = (row < C::PM_ROWS && bcol < C::PNC)
                                    ? (((nl * 3 + i) * 3 + bj) * 2 + rho) * C::NCP + el * NORB + bc
                                    : C::TRASH;
            }
        }
    }
    // N tiles starting at slot s0, processed together so that their operand
    // loads and MFMA chains interleave
    auto p_tile_group = [&](auto n_const, int s0, const TP* Xb, const TP* Ab, T* P) {
        constexpr int N = decltype(n_const)::value;
        const TP* xa[N];
        const TP* ab[N];
#pragma unroll
        for (int t = 0; t < N; ++t) {
            xa[t] = (!A_PAD || pt_aok[s0 + t]) ? Xb + pt_a[s0 + t] : sAp + ZTAIL;
            ab[t] = Ab + pt_b[s0 + t];
        }
        // two accumulators per tile (even and odd k-steps) halve the dependent
        // chain of the fp32 MFMAs; the fp64 MFMA covers its own dependency
        typename OP::Acc acc0[N], acc1[N];
#pragma unroll
        for (int t = 0; t < N; ++t) acc0[t] = acc1[t] = typename OP::Acc{};
#pragma unroll
        for (int ks = 0; ks < C::PKS; ++ks) {
#pragma unroll
            for (int t = 0; t < N; ++t) {
                TP xv = xa[t][4 * ks], bv = ab[t][4 * ks];
                if constexpr (NORB % 2 != 0) {  // the last k-step runs past u = Norb - 1
                    const bool u_ok = 2 * ks + (kk >> 1) < NORB;
                    xv = u_ok ? xv : TP(0);
                    bv = u_ok ? bv : TP(0);
                }
                if ((ks & 1) && PREC != SSE_FP64)
                    acc1[t] = OP::mma(OP::neg_if(xv, pt_neg[s0 + t]), bv, acc1[t]);
                else
                    acc0[t] = OP::mma(OP::neg_if(xv, pt_neg[s0 + t]), bv, acc0[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < N; ++t) {
            typename OP::Acc acc = acc0[t];
            if constexpr (PREC != SSE_FP64) acc += acc1[t];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                P[pt_out[s0 + t][v]] = T(acc[v]);
            }
        }
    };
    auto p_tiles = [&](int g) {
        if (g >= niter) return;
        const int np = (g % C::NCHUNK) % C::NP;
        const TP* Xb = sX + (g & 1) * C::XB;
        const TP* Ab = sAp + np * C::PSTR;
        T* P = sP + (g & 1) * C::PBS;
        // tiles in pairs, a last single one if the wave's count is odd
#pragma unroll
        for (int s0 = 0; s0 < MAXT; s0 += 2) {
            if constexpr (MAXT >= 2) {
                if (s0 + 2 <= my_count) {
                    p_tile_group(std::integral_constant<int, 2>{}, s0, Xb, Ab, P);
                    continue;
                }
            }
            if (s0 < my_count) p_tile_group(std::integral_constant<int, 1>{}, s0, Xb, Ab, P);
        }
    };

    // ---- matrix-core work of this wave: its own M-tile against every N-tile, plus
    // at most one extra (M-tile, N-tile) pair from the M-tiles past the eighth
    const bool has_own = (C::OWN == C::WAVES) || wave < C::OWN;
    const bool has_extra = wave < C::XP;
    const int own_mt = wave;
    const int ext_mt = C::WAVES + (C::XP > 0 ? wave / C::NT : 0);
    const int ext_nt = C::XP > 0 ? wave % C::NT : 0;
    auto row_info = [&](int mt, int& k, int& base, bool& neg, bool& pad) {
        const int row = 16 * mt + j16;
        pad = row >= C::MROWS;
        const int rho = row & 1, kw = row >> 1;
        k = pad ? 0 : kw / NW;
        // real embedding [[Dr, -Di], [Di, Dr]]: the (re row, im column) entry is negated
        neg = !pad && rho == 0 && kap == 1;
        base = (pad ? 0 : (kw % NW) * C::WS) + (rho ^ kap) - kap + kk;
    };
    int own_k, own_base, ext_k, ext_base;
    bool own_neg, ext_neg, own_pad, ext_pad;
    row_info(own_mt, own_k, own_base, own_neg, own_pad);
    row_info(ext_mt, ext_k, ext_base, ext_neg, ext_pad);

    // fp64 accumulators of the energy block (for fp32 operands the matrix cores
    // accumulate one K chunk in fp32, which is then added here)
    f64x4 acc[C::NT];
    f64x4 acc_x;
    auto a_ptr = [&](int k, int base, bool pad, int kp, int np) -> const T* {
        int q = k - kp;
        q += q < 0 ? NKZ : 0;
        return sD + (pad ? C::ZOFF : q * C::QS) + base + np * 36;
    };
    // The A operands of the chunk are loaded up front and the B operands one
    // k-step ahead, so LDS latency hides under the matrix instructions.
    auto mfma_chunk = [&](int g) {
        const int ch = g % C::NCHUNK, kp = ch / C::NP, np = ch % C::NP;
        const T* Pb = sP + (g & 1) * C::PBS + kk * C::NCP + j16;
        const T* Ao = a_ptr(own_k, own_base, own_pad, kp, np);
        const T* Ax = a_ptr(ext_k, ext_base, ext_pad, kp, np);
        const T* Px = Pb + 16 * ext_nt;
        // A and B operands of k-step ks + 1 are loaded while the MFMAs of ks run
        T ao[2], ax[2], bv[2][C::NT], bx[2];
        // rows of a wave without such a tile are padding rows: they read zeros
        ao[0] = Ao[0];
        ax[0] = Ax[0];
#pragma unroll
        for (int nt = 0; nt < C::NT; ++nt) bv[0][nt] = Pb[16 * nt];
        bx[0] = Px[0];
        // fp32 chunk sums: the first k-step starts from a literal zero accumulator
        // (an inline constant of the matrix instruction, no register clearing)
        typename O::Acc part[C::NT], part_x;
        const typename O::Acc zero_acc{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < C::KS; ++ks) {
            const int cur = ks & 1, nxt = cur ^ 1;
            if (ks + 1 < C::KS) {
                ao[nxt] = Ao[4 * (ks + 1)];
                ax[nxt] = Ax[4 * (ks + 1)];
#pragma unroll
                for (int nt = 0; nt < C::NT; ++nt) bv[nxt][nt] = Pb[4 * (ks + 1) * C::NCP + 16 * nt];
                bx[nxt] = Px[4 * (ks + 1) * C::NCP];
            }
            const T a = O::neg_if(ao[cur], own_neg), b = O::neg_if(ax[cur], ext_neg);
            if constexpr (PREC == SSE_FP64) {
                if (has_own) {
#pragma unroll
                    for (int nt = 0; nt < C::NT; ++nt) acc[nt] = O::mma(a, bv[cur][nt], acc[nt]);
                }
                if (has_extra) acc_x = O::mma(b, bx[cur], acc_x);
            } else {
                if (has_own) {
#pragma unroll
                    for (int nt = 0; nt < C::NT; ++nt) part[nt] = O::mma(a, bv[cur][nt], ks == 0 ? zero_acc : part[nt]);
                }
                if (has_extra) part_x = O::mma(b, bx[cur], ks == 0 ? zero_acc : part_x);
            }
        }
        if constexpr (PREC != SSE_FP64) {
#pragma unroll
            for (int nt = 0; nt < C::NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[nt][v] += (double)part[nt][v];
#pragma unroll
            for (int v = 0; v < 4; ++v) acc_x[v] += (double)part_x[v];
        }
    };

    // ---- add one V tile of energy block blk into the output ring
    // Source energy es feeds Sigma at es + w through the terms with G at E - w
    // and Sigma at es - w through those with G at E + w; FLAGS keeps either set
    // (a compile-time choice, so the usual both-branch kernel carries no test).
    constexpr bool minus = (FLAGS & kBranchMinus) != 0, plus = (FLAGS & kBranchPlus) != 0;
    constexpr bool accumulate = (FLAGS & kAccumulate) != 0;
    // Branch-free: a contribution that falls off the energy grid, or comes from a
    // padding row or column, adds 0.0 to an in-range ring entry of the tile's own
    // k set (exact, and no entry of another concurrently scattering wave).
    auto scatter_tile = [&](int blk, int mt, int nt, const f64x4& v4) {
        const int col = 16 * nt + j16;
        const bool col_ok = col < C::NCOLS;
        const int el = col_ok ? col / NORB : 0, c = col_ok ? col % NORB : 0;
        const int es = blk * EB + el;
        const bool e_ok = col_ok && es < NE;
        int pbase = (blk * EB) % C::RING + el;  // ring slot of es
        pbase -= pbase >= C::RING ? C::RING : 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * mt + O::row_of(lane, v);
            const bool row_ok = row < C::MROWS, ok = e_ok && row_ok;
            // padding rows (last M-tile only) take the last real row's momentum,
            // which is in that tile's k set
            const int rho = row & 1, kw = row_ok ? row >> 1 : C::MROWS / 2 - 1, k = kw / NW, w = kw % NW + 1;
            const int off = (k * NORB + c) * 2 + rho;
            int plo = pbase - w, phi = pbase + w;
            plo += plo < 0 ? C::RING : 0;
            phi -= phi >= C::RING ? C::RING : 0;
            atomicAdd(&sR[plo * C::RP + off], (ok && plus && es - w >= 0) ? v4[v] : 0.0);
            atomicAdd(&sR[phi * C::RP + off], (ok && minus && es + w < NE) ? v4[v] : 0.0);
        }
    };
    constexpr ScatterPlan<C> plan{};
    auto scatter = [&](int blk, int phase) {
        if (has_own && plan.own_phase[wave] == phase) {
#pragma unroll
            for (int nt = 0; nt < C::NT; ++nt) scatter_tile(blk, own_mt, nt, acc[nt]);
        }
        if (has_extra && plan.ext_phase[wave] == phase) scatter_tile(blk, ext_mt, ext_nt, acc_x);
    };

    // ---- scale by alpha and store output planes [e_lo, e_hi); clear their ring slots
    auto write_planes = [&](int e_lo, int e_hi) {
        if (e_lo < 0) e_lo = 0;
        if (e_hi > NE) e_hi = NE;
        const int per = NKZ * NORB;
        for (int x = tid; x < (e_hi - e_lo) * per; x += C::THREADS) {
            const int e = e_lo + x / per;
            const int kc = x % per, k = kc / NORB, c = kc % NORB;
            double* slot = sR + (e % C::RING) * C::RP + kc * 2;
            const cd v{slot[0], slot[1]};
            slot[0] = 0.0;
            slot[1] = 0.0;
            const int64_t o = (((int64_t)k * NE + e) * na + a) * C::NN + r * NORB + c;
            cd out = cmul(alpha, v);
            if constexpr (accumulate) {
                const cd old = cload(S, o);
                out = cd{old.re + out.re, old.im + out.im};
            }
            cstore(S, o, out);
        }
    };

    // ---- the two waves of a SIMD (w and w+4) run opposite phases: waves 0-3
    // issue their matrix work first and form P and X afterwards, waves 4-7 form
    // P and X (from G loads issued in the previous chunk) first, so the vector
    // work of one wave runs under the matrix work of the other.  Every phase has
    // one call site, which keeps the accumulators in place across the loop.
    const bool mfma_first = wave < 4;

    // ---- prologue: X for chunks 0 and 1, P for chunk 0
    __syncthreads();
    gather_g(0);
    finish_x(0);
    __syncthreads();
    gather_g(1);
    p_tiles(0);
    finish_x(1);
    if (!mfma_first) gather_g(2);
    __syncthreads();

    // ---- main loop: energy blocks, K chunks inside, one barrier per chunk
    for (int blk = 0; blk < nblk; ++blk) {
#pragma unroll
        for (int nt = 0; nt < C::NT; ++nt) acc[nt] = f64x4{0.0, 0.0, 0.0, 0.0};
        acc_x = f64x4{0.0, 0.0, 0.0, 0.0};
        for (int ch = 0; ch < C::NCHUNK; ++ch) {
            const int g = blk * C::NCHUNK + ch;
            if (!mfma_first) {
                finish_x(g + 2);  // G for chunk g+2 was gathered during chunk g-1
                p_tiles(g + 1);
            }
            gather_g(mfma_first ? g + 2 : g + 3);  // loads in flight under the matrix work
            mfma_chunk(g);
            if (mfma_first) {
                p_tiles(g + 1);
                finish_x(g + 2);
            }
            __syncthreads();
        }
        for (int ph = 0; ph < plan.nphase; ++ph) {
            scatter(blk, ph);
            __syncthreads();
        }
        write_planes(blk * EB - NW, (blk + 1) * EB - NW);
    }
    write_planes(nblk * EB - NW, NE);
}

template <int NORB, int NKZ, int NW, int NB, int EB, int PREC, int FLAGS, bool HBA>
static hipError_t launch_fwd_flags(const Dims& d, const double* G, const double* D, const double* A, const double* B,
                                   const int32_t* nbr, cd alpha, double* S, hipStream_t stream) {
    using C = Fwd64<NORB, NKZ, NW, NB, EB, PREC, HBA>;
    auto kern = fwd_mfma_kernel<NORB, NKZ, NW, NB, EB, PREC, FLAGS, HBA>;
    // set on every launch (cheap): the attribute is per device, and a process-wide
    // flag would race between host threads
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)C::LDS_BYTES);
    if (e != hipSuccess) return e;
    // The Norb row workgroups of an atom start together and share its G blocks in
    // L2 while they stay within a few chunks of each other; over a long launch
    // they drift apart (each compute unit runs its workgroups one after another
    // and their durations vary) and the sharing is lost.  Launches of about
    // twelve rounds of workgroups (304 atoms on 256 compute units at Norb = 10)
    // start every atom's rows together again; the boundaries cost no measurable
    // time at the device workload.
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t na8 = ((d.na + 7) / 8) * 8;
    const int64_t batch = std::max<int64_t>(8, (int64_t)12 * cus / NORB / 8 * 8);
    for (int64_t a0 = 0; a0 < na8; a0 += batch) {
        const int64_t atoms = std::min(batch, na8 - a0);
        hipLaunchKernelGGL(kern, dim3((unsigned)(atoms * NORB)), dim3(C::THREADS), C::LDS_BYTES, stream, d, G, D, A, B,
                           nbr, alpha, S, a0);
    }
    return hipGetLastError();
}

// the branch sets with a kernel instance: both (one pass), and the two passes
// of the signed form (E - w terms written, E + w terms added)
template <int NORB, int NKZ, int NW, int NB, int EB, int PREC, bool HBA>
static hipError_t launch_fwd(const Dims& d, const double* G, const double* D, const double* A, const double* B,
                             const int32_t* nbr, cd alpha, double* S, hipStream_t stream, int flags) {
    constexpr int kBoth = kBranchMinus | kBranchPlus, kPlusAdd = kBranchPlus | kAccumulate;
    if (flags == kBoth)
        return launch_fwd_flags<NORB, NKZ, NW, NB, EB, PREC, kBoth, HBA>(d, G, D, A, B, nbr, alpha, S, stream);
    if (flags == kBranchMinus)
        return launch_fwd_flags<NORB, NKZ, NW, NB, EB, PREC, kBranchMinus, HBA>(d, G, D, A, B, nbr, alpha, S, stream);
    if (flags == kPlusAdd)
        return launch_fwd_flags<NORB, NKZ, NW, NB, EB, PREC, kPlusAdd, HBA>(d, G, D, A, B, nbr, alpha, S, stream);
    return hipErrorInvalidValue;
}

bool fwd_mfma_specialised(const Dims& d) {
    if (d.ne >= (int64_t(1) << 28)) return false;  // 32-bit chunk indices
    return (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 4) || (d.norb == 4 && d.nkz == 3 && d.nw == 2 && d.nb == 4) ||
           (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 3) || (d.norb == 12 && d.nkz == 7 && d.nw == 10 && d.nb == 4);
}

// Norb = 12 (the paper's orbital count) fits the LDS with blocks of 4 source
// energies, for fp64 and fp32 operands and grad H^H as the right factor only
// (a stored grad H_ba table, or the 16-bit layout, would not fit)
bool fwd_mfma_supports(const Dims& d, int precision, bool hba) {
    if (!fwd_mfma_specialised(d)) return false;
    if (d.norb == 12) return (precision == SSE_FP64 || precision == SSE_FP32) && !hba;
    return true;
}

// energy blocks of 8 source energies; with a stored grad H_ba the fp64 form
// takes blocks of 4, which leaves LDS room for the second right-factor table
template <int NORB, int NKZ, int NW, int NB, int PREC>
static hipError_t launch_shape(const Dims& d, const double* G, const double* D, const double* A, const double* B,
                               const int32_t* nbr, cd alpha, double* S, hipStream_t stream, int flags) {
    if (!B) return launch_fwd<NORB, NKZ, NW, NB, 8, PREC, false>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    return launch_fwd<NORB, NKZ, NW, NB, PREC == SSE_FP64 ? 4 : 8, PREC, true>(d, G, D, A, B, nbr, alpha, S, stream,
                                                                                 flags);
}

template <int PREC>
static hipError_t dispatch_fwd(const Dims& d, const double* G, const double* D, const double* A, const double* B,
                               const int32_t* nbr, cd alpha, double* S, hipStream_t stream, int flags) {
    if (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 4)
        return launch_shape<10, 7, 10, 4, PREC>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 3)
        return launch_shape<10, 7, 10, 3, PREC>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (d.norb == 4 && d.nkz == 3 && d.nw == 2 && d.nb == 4)
        return launch_shape<4, 3, 2, 4, PREC>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (d.norb == 12 && d.nkz == 7 && d.nw == 10 && d.nb == 4 && !B)
        return launch_fwd<12, 7, 10, 4, 4, PREC, false>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    return hipErrorInvalidValue;
}

hipError_t launch_fwd_mfma(const Dims& d, int precision, const double* G, const double* D, const double* A,
                           const double* B, const int32_t* nbr, cd alpha, double* S, hipStream_t stream, int flags) {
    if (precision == SSE_FP64) return dispatch_fwd<SSE_FP64>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (precision == SSE_FP32) return dispatch_fwd<SSE_FP32>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (precision == SSE_FP16X2 || precision == SSE_BF16X2 || precision == SSE_FP16 || precision == SSE_FP16_UNSCALED)
        return launch_fwd_h16(d, precision, G, D, A, B, nbr, alpha, S, stream, flags);
    return hipErrorInvalidValue;
}

}  // namespace sse
