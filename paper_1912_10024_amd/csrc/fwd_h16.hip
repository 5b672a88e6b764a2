// Matrix-core forward kernel of the scattering self-energy (Eq. 3) with split
// 16-bit operands: fp16 hi + lo after power-of-two normalisation (the paper's
// normalised half precision, Sec. "Mixed-Precision Computation", with
// compensation) or bfloat16 hi + lo (fp32's exponent range, no scaling).
//
// Same regrouping as the fp64 kernel (fission of Sec. "Dataflow
// Optimizations"), per atom a and output row r:
//
//   P[k',E',n,i,j][r][c] = (grad_i H_{a,n} . G[k',E',nbr[a,n],0] . grad_j H_{a,n}^H)[r][c]
//   V[(k,w),(E',c)]      = sum_{k',n,i,j} D[(k-k') mod Nkz, w-1, a, n, i, j] * P[k',E',n,i,j][r][c]
//   Sigma[k,E,a][r][c]   = alpha * sum_w ( V[(k,w),(E-w,c)] + V[(k,w),(E+w,c)] )
//
// Every dense product runs on the 16x16x32 16-bit matrix instructions, whose
// lanes carry eight 16-bit values per operand.  A value x is split as x ~ hi +
// lo (hi = r(x), lo = r(x - hi)).  Two operand schemes keep all four partial
// products of every element (exact in fp32, summed in fp32):
//  - main GEMM, four K elements per lane and two instructions: B holds (x0h,
//    x0l, x1h, x1l, x2h, x2l, x3h, x3l) as stored in LDS (one 16-byte load), A
//    holds (y0h, y0h, y1h, y1h, y2h, y2h, y3h, y3h) in the first instruction and
//    the lo parts in the second, so the two give sum_m (y_mh + y_ml) x_m; LDS
//    keeps the hi and lo parts of A packed (8 bytes per four elements each) and
//    byte permutes rebuild the operands, once per K step for all N-tiles;
//  - P tiles, two K elements per lane: M form (x1h, x1l, x2h, x2l, x1h, x1l,
//    x2h, x2l) times P form (y1h, y1h, y2h, y2h, y1l, y1l, y2l, y2l) slot by slot
//    is x1 y1 + x2 y2; LDS keeps 8 bytes per pair for each.
//
// Work decomposition: one workgroup of 8 waves per (atom, output row r), energy
// blocks of EB = 8 source energies, one K chunk per momentum k' holding all Nb
// neighbours: K = Nb * 9 complex entries (n, i, j), in groups of eight with one
// real component per lane group.  Main GEMM per chunk: rows (k, w, re/im),
// columns (E', c); its A operand comes from three planes of the per-atom D
// table, Re D, Im D and -Im D, so that the real embedding [[Dr, -Di], [Di, Dr]]
// needs no sign changes; its B operand is the P chunk.  The P chunk itself is a
// second GEMM per neighbour: rows (i, E'), K = (u, re/im) of X = grad_i H . G
// (row r), columns (j, c, re/im) against the embedding of conj(grad_j H) with
// the signs placed in the static table ((Re, Im) -> (Ar, Ai) for the real
// column and (-Ai, Ar) for the imaginary one; with a stored grad_j H_ba, B =
// Bba_j[u][c] takes the place of conj(A_j[c][u])).  X rows are formed in fp64
// on the vector ALUs from the gathered G columns, normalised (fp16) and split
// once.
//
// Pipeline per chunk (one barrier): form the P chunk of the next chunk from the
// X rows in LDS, form the X rows of the chunk after that from G columns
// gathered into registers one chunk earlier, run the main GEMM on the P chunk
// in LDS, gather the G columns of a later chunk.  The 16-bit matrix
// instructions of one wave run while the other wave of the SIMD issues vector
// work.  Each chunk's fp32 sums are unscaled
// and added to fp64 accumulators; the (w, +/-) stencil adds them into an fp64
// output ring in LDS in conflict-free phases (bitwise reproducible).
#include "fwd_common.h"
#include "sse_kernels.h"

namespace sse {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Operand arithmetic per precision: the 16-bit matrix instruction, the split
// of an fp32 value into its (hi, lo) word, whether the lo terms are kept (LO)
// and whether the operands are normalised by powers of two (NORM)
template <int PREC>
struct Split16;
template <>
struct Split16<SSE_FP16X2> {
    static constexpr bool LO = true, NORM = true;
    static __device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0,
                                                      0);
    }
    // (hi, lo) of x as one word, hi in the low half; x - hi is exact in fp32
    static __device__ __forceinline__ unsigned split(float x) {
        const _Float16 h = (_Float16)x;
        const _Float16 l = (_Float16)(x - (float)h);
        return __builtin_bit_cast(unsigned, f16x2{h, l});
    }
};
template <>
struct Split16<SSE_BF16X2> {
    static constexpr bool LO = true, NORM = false;
    static __device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                       0, 0);
    }
    static __device__ __forceinline__ unsigned split(float x) {
        const __bf16 h = (__bf16)x;  // round to nearest even
        const __bf16 l = (__bf16)(x - (float)h);
        return (unsigned)__builtin_bit_cast(unsigned short, h) | ((unsigned)__builtin_bit_cast(unsigned short, l) << 16);
    }
};
// The paper's scheme without compensation: one fp16 term per operand (lo = 0,
// so the P tiles' lo products add zeros and the main GEMM drops its lo
// instruction), after the normalisation of the two-term form
template <>
struct Split16<SSE_FP16> {
    static constexpr bool LO = false, NORM = true;
    static __device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
        return Split16<SSE_FP16X2>::mma(a, b, c);
    }
    static __device__ __forceinline__ unsigned split(float x) {
        return (unsigned)__builtin_bit_cast(unsigned short, (_Float16)x);
    }
};
// ... and without the normalisation: magnitudes beyond the fp16 range are
// clamped to its largest finite value, smaller ones round to fp16 as they are
template <>
struct Split16<SSE_FP16_UNSCALED> {
    static constexpr bool LO = false, NORM = false;
    static __device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
        return Split16<SSE_FP16X2>::mma(a, b, c);
    }
    static __device__ __forceinline__ unsigned split(float x) {
        return Split16<SSE_FP16>::split(fminf(fmaxf(x, -65504.0f), 65504.0f));
    }
};

// P-tile operands from their 8-byte LDS form: M form (w1, w2, w1, w2), P form
// with every half duplicated
__device__ __forceinline__ u32x4 m_operand(uint2 w) { return u32x4{w.x, w.y, w.x, w.y}; }
__device__ __forceinline__ u32x4 dup_halves(unsigned a, unsigned b) {
    return u32x4{__builtin_amdgcn_perm(a, a, 0x01000100u), __builtin_amdgcn_perm(a, a, 0x03020302u),
                 __builtin_amdgcn_perm(b, b, 0x01000100u), __builtin_amdgcn_perm(b, b, 0x03020302u)};
}
__device__ __forceinline__ u32x4 p_operand(uint2 w) { return dup_halves(w.x, w.y); }
// main-GEMM A operands of four elements from (hi0|hi1, hi2|hi3, lo0|lo1, lo2|lo3)
__device__ __forceinline__ u32x4 hi_operand(uint4 q) { return dup_halves(q.x, q.y); }
__device__ __forceinline__ u32x4 lo_operand(uint4 q) { return dup_halves(q.z, q.w); }
__device__ __forceinline__ u32x4 as_u32x4(uint4 q) { return u32x4{q.x, q.y, q.z, q.w}; }
// x rounded to fp32 and kept there: without the (empty) register constraint the
// compiler fuses the fp64 -> fp32 -> 16-bit conversions of a split into one
// fp64 -> fp16 conversion, which has no instruction and takes ~30 integer ops
__device__ __forceinline__ float to_f32(double x) {
    float f = (float)x;
    __asm__("" : "+v"(f));
    return f;
}
// P form of two values from their (hi | lo << 16) words
__device__ __forceinline__ uint2 p_form(unsigned m1, unsigned m2) {
    return make_uint2((m1 & 0xffffu) | (m2 << 16), (m1 >> 16) | (m2 & 0xffff0000u));
}
// packed hi and lo parts of four values (the main-GEMM A table)
__device__ __forceinline__ uint4 hl_quad(const unsigned w[4]) {
    const uint2 a = p_form(w[0], w[1]), b = p_form(w[2], w[3]);
    return make_uint4(a.x, b.x, a.y, b.y);
}

}  // namespace

template <int NORB, int NKZ, int NW, int NB, int EB>
struct H16Cfg {
    static constexpr int WAVES = 8, THREADS = 64 * WAVES;
    static constexpr int NN = NORB * NORB;
    static constexpr int NWV = NW;
    // main GEMM: rows (k, w, re/im), columns (E', c)
    static constexpr int MROWS = 2 * NKZ * NW;
    static constexpr int MT = (MROWS + 15) / 16;
    static constexpr int NCOLS = EB * NORB;
    static constexpr int NT = (NCOLS + 15) / 16;
    // K of one chunk: complex entries e = 9 n + 3 i + j in groups of eight (zero
    // padded); a K step takes one group, lane group kk holds entries 8 t + 4 (kk/2)
    // + m (m < 4) of component kk & 1 (Re or Im column of P)
    static constexpr int NENT = NB * 9;
    static constexpr int NG = (NENT + 7) / 8;
    // D table (16-byte units): per (q, w) the planes Re D, Im D, -Im D, each with
    // 2 NG quads of packed hi and lo parts; an odd stride spreads the rows of an
    // operand load over the banks
    static constexpr int DQW = 6 * NG + 1;
    static constexpr int ZOFF = NKZ * NW * DQW;  // zero quads read by padding rows
    static constexpr int L_D = ZOFF + 2 * NG + 2;
    // P chunk (16-byte units) [row 4 t + kk][column (E', c)]: (hi | lo << 16) of four
    // entries, two buffers; the unit after each buffer takes the padding results
    // of the P tiles
    static constexpr int NCP = NT * 16 + 1;  // odd: the rows of a unit's Re and Im hit different banks
    static constexpr int TRASH = 4 * NG * NCP;
    static constexpr int PBS = TRASH + EB * NORB;  // spare units: four stores at a stride of 4 Norb words
    static constexpr int L_P = 2 * PBS;
    // P tiles, one GEMM per neighbour: rows (E', i), K pairs u (Re, Im), columns (j, c, re/im)
    static constexpr int PM = EB * 3;
    static constexpr int PMT = (PM + 15) / 16;
    static constexpr int PKS = (NORB + 3) / 4;    // K steps; pairs u >= Norb read zeros
    static constexpr int PN = 2 * 3 * NORB;
    static constexpr int PNT = (PN + 15) / 16;
    static constexpr int HCOLS = PNT * 16;
    static constexpr int HZ = NB * NORB * HCOLS;   // a zero pair
    static constexpr int L_H = HZ + 2;             // conj(grad H) embedding [n][u][col], P form
    static constexpr int XRS = PM + 1;             // odd stride of the (n, u) row blocks (bank spread)
    static constexpr int XB = NB * NORB * XRS;     // one buffer of X rows [n][u][i EB + E'], M form
    static constexpr int XZ = 2 * XB;              // a zero pair read by padding rows and pairs
    static constexpr int L_X = 2 * XB + 2;
    static constexpr int UNITS = NB * PNT;         // P-tile units (neighbour, column tile)
    static constexpr int MAXU = (UNITS + WAVES - 1) / WAVES;
    // fp64: row r of grad H [n][i][t] for the X rows, the output ring, scale slots
    static constexpr int L_AR = NB * 3 * NORB * 2;
    static constexpr int RING = EB + 2 * NW;
    static constexpr int RP = NKZ * NORB * 2;
    static constexpr int L_R = RING * RP;
    static constexpr int L_S = 4 * EB > WAVES ? 4 * EB : WAVES;
    static constexpr int U8 = 2 * (L_D + L_P) + L_H + L_X;  // 8-byte units of the 16-bit tables
    static constexpr size_t LDS_BYTES = 8 * (size_t)(U8 + L_AR + L_R + L_S);
    // wave ownership of main-GEMM tiles: a whole M-tile per wave, the M-tiles past
    // the eighth dealt out one (M-tile, N-tile) pair per wave
    static constexpr int OWN = MT < WAVES ? MT : WAVES;
    static constexpr int XP = MT > WAVES ? (MT - WAVES) * NT : 0;
    static constexpr int X_LANES = NB * NORB;  // X rows: lane (n, u) of wave E'
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
    static_assert(EB == WAVES, "wave w forms the X rows of source energy w");
    static_assert(PM <= 2 * 16 && EB == 8, "P-tile rows (i, E'): i = 2 mt + kk / 2, E' = 4 (kk & 1) + v");
    static_assert(X_LANES <= 64, "one lane per (neighbour, column u)");
    static_assert(XP <= WAVES, "at most one extra (M-tile, N-tile) pair per wave");
    static_assert(NKZ <= 32, "momentum sets of a tile fit a 32-bit mask");
};

template <int NORB, int NKZ, int NW, int NB, int EB, int PREC, int FLAGS>
__global__ __launch_bounds__(512) void fwd_h16_kernel(Dims d, const double* __restrict__ G,
                                                      const double* __restrict__ Dg, const double* __restrict__ Ag,
                                                      const double* __restrict__ Bg, const int32_t* __restrict__ nbr,
                                                      cd alpha, double* __restrict__ S) {
    using C = H16Cfg<NORB, NKZ, NW, NB, EB>;
    using O = Split16<PREC>;
    constexpr bool NORM = O::NORM;
    extern __shared__ double lds[];
    uint4* sD = reinterpret_cast<uint4*>(lds);
    uint4* sP = sD + C::L_D;
    uint2* sH = reinterpret_cast<uint2*>(sP + C::L_P);
    uint2* sX = sH + C::L_H;
    double* sAr = lds + C::U8;
    double* sR = sAr + C::L_AR;
    double* sS = sR + C::L_R;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // XCD-aware mapping: the Norb workgroups of one atom share its D, grad H and
    // neighbour G blocks, so they get block ids that land on the same XCD.
    const int64_t bid = blockIdx.x;
    const int r = (int)((bid >> 3) % NORB);
    const int64_t a = ((bid >> 3) / NORB) * 8 + (bid & 7);
    if (a >= d.na) return;  // uniform for the whole workgroup, before any barrier

    // ---- fp16: per-atom power-of-two normalisation of D (largest part below 2^7)
    // and grad H (below 2; with a stored grad H_ba, over both factors), from
    // workgroup maxima
    double sc_d = 1.0, sc_h = 1.0, inv_base = 1.0;
    if constexpr (NORM) {
        auto block_max = [&](double m) {
            for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
            __syncthreads();
            if (lane == 0) sS[wave] = m;
            __syncthreads();
            double v = sS[0];
            for (int w = 1; w < C::WAVES; ++w) v = fmax(v, sS[w]);
            return v;
        };
        double md = 0.0, mh = 0.0;
        for (int x = tid; x < NKZ * NW * NB * 9; x += C::THREADS) {
            const int ij = x % 9, n = (x / 9) % NB, w = (x / (9 * NB)) % NW, q = x / (9 * NB * NW);
            const cd v = cload(Dg, off_D(d, q, w, a, n) + ij);
            md = fmax(md, fmax(fabs(v.re), fabs(v.im)));
        }
        for (int x = tid; x < NB * 3 * C::NN; x += C::THREADS) {
            const cd v = cload(Ag, off_A(d, a, 0, 0) + x);
            mh = fmax(mh, fmax(fabs(v.re), fabs(v.im)));
            if (Bg) {
                const cd b = cload(Bg, off_A(d, a, 0, 0) + x);
                mh = fmax(mh, fmax(fabs(b.re), fabs(b.im)));
            }
        }
        sc_d = pow2_scale(block_max(md), 7);
        sc_h = pow2_scale(block_max(mh), 1);
        inv_base = 1.0 / (sc_d * sc_h * sc_h);
    }

    // ---- clear the tables (padding rows, columns and K pairs read zeros), then stage
    for (int x = tid; x < C::U8; x += C::THREADS) reinterpret_cast<uint2*>(lds)[x] = make_uint2(0u, 0u);
    for (int x = tid; x < C::L_R; x += C::THREADS) sR[x] = 0.0;
    __syncthreads();
    // D: planes Re D, Im D, -Im D per (q, w), quads of consecutive entries (n, i, j)
    for (int x = tid; x < NKZ * NW * 2 * C::NG; x += C::THREADS) {
        const int hq = x % (2 * C::NG), qw = x / (2 * C::NG);
        unsigned re[4], im[4], nim[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int e = 4 * hq + m;
            cd v{0.0, 0.0};
            if (e < C::NENT) v = cload(Dg, off_D(d, qw / NW, qw % NW, a, e / 9) + e % 9);
            re[m] = O::split(to_f32(v.re * sc_d));
            im[m] = O::split(to_f32(v.im * sc_d));
            nim[m] = im[m] ^ 0x80008000u;  // -Im: both halves negated
        }
        uint4* o = sD + qw * C::DQW + hq;
        o[0] = hl_quad(re);
        o[2 * C::NG] = hl_quad(im);
        o[4 * C::NG] = hl_quad(nim);
    }
    // row r of grad H for the X rows (fp64)
    for (int x = tid; x < NB * 3 * NORB; x += C::THREADS) {
        const int ni = x / NORB, t = x % NORB;
        const cd v = cload(Ag, off_A(d, a, ni / 3, ni % 3) + r * NORB + t);
        sAr[2 * x] = v.re * sc_h;
        sAr[2 * x + 1] = v.im * sc_h;
    }
    // embedding of the right factor B = grad_j H_ba for the P tiles, B[u][c] =
    // conj(A_j[c][u]) or the stored block: K pair u = (Re, Im) of X[u]; column
    // (j, c, 0) takes (Br, -Bi) (real part of X . B), column (j, c, 1) takes
    // (Bi, Br) (imaginary part)
    for (int x = tid; x < NB * NORB * C::PN; x += C::THREADS) {
        const int col = x % C::PN, u = (x / C::PN) % NORB, n = x / (C::PN * NORB);
        const int comp = col & 1, jc = col >> 1, c = jc % NORB;
        double br, bi;
        if (Bg) {
            const cd v = cload(Bg, off_A(d, a, n, jc / NORB) + u * NORB + c);
            br = v.re * sc_h;
            bi = v.im * sc_h;
        } else {
            const cd v = cload(Ag, off_A(d, a, n, jc / NORB) + c * NORB + u);
            br = v.re * sc_h;
            bi = -v.im * sc_h;
        }
        const double b0 = comp ? bi : br, b1 = comp ? br : -bi;
        sH[(n * NORB + u) * C::HCOLS + col] = p_form(O::split(to_f32(b0)), O::split(to_f32(b1)));
    }

    // chunk and energy indices fit 32 bits: the dispatcher admits ne < 2^28
    const int NE = (int)d.ne;
    const int nblk = (NE + EB - 1) / EB;
    const int niter = nblk * NKZ;
    const int kk = lane >> 4, j16 = lane & 15;

    // ---- X rows, step 1: lane (n, u) of wave E' gathers column u of G[k', E', nbr[a,n], 0]
    const bool x_lane = lane < C::X_LANES;
    const int x_n = x_lane ? lane / NORB : 0, x_u = lane % NORB;
    const int64_t na = d.na;
    const int32_t xb = x_lane ? nbr[a * NB + x_n] : -1;
    const bool b_ok = x_lane && xb >= 0 && xb < na;  // an entry outside [0, na) contributes zero
    const int64_t e_step = 2 * d.gs * C::NN * na, kp_step = e_step * NE;
    const int64_t b_off = b_ok ? 2 * d.gs * C::NN * (int64_t)xb + 2 * x_u : 0;
    cd gv[NORB];
    bool g_ok = false;
    // branch-free: an invalid lane loads from the start of G and finish_x writes zero for it
    auto gather_g = [&](int g) {
        const int gg = g < niter ? g : 0;
        const int e = (gg / NKZ) * EB + wave;
        g_ok = g < niter && b_ok && e < NE;
        const double* Gb = G + (g_ok ? b_off + (gg % NKZ) * kp_step + (int64_t)e * e_step : 0);
#pragma unroll
        for (int t = 0; t < NORB; ++t) gv[t] = cd{Gb[2 * t * NORB], Gb[2 * t * NORB + 1]};
    };
    // ---- X rows, step 2: X_i[u] = sum_t gradH[n][i][r][t] G[t][u] for i = 0..2 (fp64);
    // fp16: the X rows of one source energy (one wave) are normalised by a power of
    // two (largest part below 2^XT, which keeps every P entry below 2^14); the
    // inverse of all scale factors of the chunk's column goes to LDS
    constexpr int XT = 14 - ceil_log2(4 * NORB);
    auto finish_x = [&](int g) {
        if (g >= niter) return;
        cd x[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double* Ar = sAr + 2 * ((x_n * 3 + i) * NORB);
            x[i] = cd{0.0, 0.0};
#pragma unroll
            for (int t = 0; t < NORB; ++t) cfma(x[i], cd{Ar[2 * t], Ar[2 * t + 1]}, gv[t]);
            if (!g_ok) x[i] = cd{0.0, 0.0};
        }
        int shift = 0;
        if constexpr (NORM) {
            double m = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) m = fmax(m, fmax(fabs(x[i].re), fabs(x[i].im)));
            int e = -4000;
            if (m > 0.0) frexp(m, &e);
            e = wave_max(e);
            shift = e == -4000 ? 0 : XT - e;
            if (lane == 0) sS[(g & 3) * EB + wave] = ldexp(inv_base, -shift);
        }
        if (!x_lane) return;
        uint2* X = sX + (g & 1) * C::XB + (x_n * NORB + x_u) * C::XRS + wave;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double re = x[i].re, im = x[i].im;
            if constexpr (NORM) {
                re = ldexp(re, shift);
                im = ldexp(im, shift);
            }
            X[i * EB] = make_uint2(O::split(to_f32(re)), O::split(to_f32(im)));
        }
    };

    // ---- P tiles: units (neighbour n, column tile) dealt round robin, each unit
    // runs its PMT row tiles (rows i EB + E') against one conj(grad H) operand per
    // K step
    auto p_tiles = [&](int g) {
        if (g >= niter) return;
        const uint2* Xb = sX + (g & 1) * C::XB;
        uint32_t* P = reinterpret_cast<uint32_t*>(sP + (g & 1) * C::PBS);
        f32x4 acc[C::MAXU][C::PMT];
#pragma unroll
        for (int ui = 0; ui < C::MAXU; ++ui) {
            const int unit = wave + C::WAVES * ui;
            if (unit >= C::UNITS) break;  // uniform per wave
            const int n = unit / C::PNT, nt = unit % C::PNT;
#pragma unroll
            for (int mt = 0; mt < C::PMT; ++mt) acc[ui][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < C::PKS; ++s) {
                const int u = 4 * s + kk;
                const bool u_ok = 4 * s + 3 < NORB || u < NORB;
                const uint2* hp = u_ok ? sH + (n * NORB + u) * C::HCOLS + 16 * nt + j16 : sH + C::HZ;
                const u32x4 hb = p_operand(*hp);
#pragma unroll
                for (int mt = 0; mt < C::PMT; ++mt) {
                    const int row = 16 * mt + j16;
                    const uint2* xp = (u_ok && row < C::PM) ? Xb + (n * NORB + u) * C::XRS + row : sX + C::XZ;
                    acc[ui][mt] = O::mma(m_operand(*xp), hb, acc[ui][mt]);
                }
            }
        }
        // P entry e = 9 n + 3 i + j, component re/im, of column (E', c) into its
        // slot of the 16-byte unit (row 4 (e/8) + 2 ((e/4)&1) + comp); a lane's four
        // results are consecutive E' of one i; padding rows and columns write the
        // spare unit.  The stores follow all the products of the wave's units, so
        // the matrix pipeline drains once.
#pragma unroll
        for (int ui = 0; ui < C::MAXU; ++ui) {
            const int unit = wave + C::WAVES * ui;
            if (unit >= C::UNITS) break;
            const int n = unit / C::PNT, nt = unit % C::PNT;
            const int col = 16 * nt + j16;
            const int comp = col & 1, jc = col >> 1, j = jc / NORB, c = jc % NORB;
#pragma unroll
            for (int mt = 0; mt < C::PMT; ++mt) {
                const int i = 2 * mt + (kk >> 1);
                const int e = n * 9 + 3 * i + j;
                const int prow = 4 * (e >> 3) + 2 * ((e >> 2) & 1) + comp;
                const bool ok = i < 3 && col < C::PN;
                uint32_t* dst = P + (ok ? (prow * C::NCP + 4 * (kk & 1) * NORB + c) * 4 + (e & 3) : 4 * C::TRASH);
#pragma unroll
                for (int v = 0; v < 4; ++v) dst[v * 4 * NORB] = O::split(acc[ui][mt][v]);
            }
        }
    };

    // ---- main GEMM: this wave's M-tile against every N-tile, plus at most one
    // extra (M-tile, N-tile) pair from the M-tiles past the eighth
    const bool has_own = (C::OWN == C::WAVES) || wave < C::OWN;
    const bool has_extra = wave < C::XP;
    const int own_mt = wave;
    const int ext_mt = C::WAVES + (C::XP > 0 ? wave / C::NT : 0);
    const int ext_nt = C::XP > 0 ? wave % C::NT : 0;
    // A operand of a row (k, w, rho): the quad of entries (t, kk/2), component
    // kap = kk & 1, of the D plane that the real embedding puts there
    auto row_info = [&](int mt, int& k, int& base, bool& pad) {
        const int row = 16 * mt + j16;
        pad = row >= C::MROWS;
        const int rho = row & 1, kw = row >> 1, kap = kk & 1, half = kk >> 1;
        k = pad ? 0 : kw / NW;
        const int plane = rho == 0 ? (kap == 0 ? 0 : 2) : (kap == 0 ? 1 : 0);
        base = pad ? C::ZOFF + half : (kw % NW) * C::DQW + plane * 2 * C::NG + half;
    };
    int own_k, own_base, ext_k, ext_base;
    bool own_pad, ext_pad;
    row_info(own_mt, own_k, own_base, own_pad);
    row_info(ext_mt, ext_k, ext_base, ext_pad);
    auto a_ptr = [&](int k, int base, bool pad, int kp) -> const uint4* {
        int q = k - kp;
        q += q < 0 ? NKZ : 0;
        return sD + (pad ? 0 : q * NW * C::DQW) + base;
    };

    f64x4 acc[C::NT];
    f64x4 acc_x;
    // per K step: the hi and lo A operands of the wave's rows against the B operand
    // of every N-tile; the operands of step t + 1 are loaded while the products of
    // step t run
    auto mfma_chunk = [&](int g) {
        const int kp = g % NKZ;
        const uint4* Pb = sP + (g & 1) * C::PBS + kk * C::NCP + j16;
        const uint4* Ao = a_ptr(own_k, own_base, own_pad, kp);
        const uint4* Ax = a_ptr(ext_k, ext_base, ext_pad, kp);
        const uint4* Px = Pb + 16 * ext_nt;
        uint4 ao[2], ax[2], bv[2][C::NT], bx[2];
        ao[0] = Ao[0];
        ax[0] = Ax[0];
#pragma unroll
        for (int nt = 0; nt < C::NT; ++nt) bv[0][nt] = Pb[16 * nt];
        bx[0] = Px[0];
        // each chunk's sums start from a literal zero accumulator
        f32x4 part[C::NT], part_x;
        const f32x4 zero_acc{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < C::NG; ++t) {
            const int cur = t & 1, nxt = cur ^ 1;
            if (t + 1 < C::NG) {
                ao[nxt] = Ao[2 * (t + 1)];
                ax[nxt] = Ax[2 * (t + 1)];
#pragma unroll
                for (int nt = 0; nt < C::NT; ++nt) bv[nxt][nt] = Pb[4 * (t + 1) * C::NCP + 16 * nt];
                bx[nxt] = Px[4 * (t + 1) * C::NCP];
            }
            if (has_own) {
                const u32x4 ah = hi_operand(ao[cur]), al = lo_operand(ao[cur]);
#pragma unroll
                for (int nt = 0; nt < C::NT; ++nt)
                    part[nt] = O::mma(ah, as_u32x4(bv[cur][nt]), t == 0 ? zero_acc : part[nt]);
                if constexpr (O::LO) {
#pragma unroll
                    for (int nt = 0; nt < C::NT; ++nt) part[nt] = O::mma(al, as_u32x4(bv[cur][nt]), part[nt]);
                }
            }
            if (has_extra) {
                part_x = O::mma(hi_operand(ax[cur]), as_u32x4(bx[cur]), t == 0 ? zero_acc : part_x);
                if constexpr (O::LO) part_x = O::mma(lo_operand(ax[cur]), as_u32x4(bx[cur]), part_x);
            }
        }
        // the chunk (one qz per output momentum) goes into the fp64 sums; fp16:
        // with the inverse scale of the lane's column (source energy)
        auto inv_of = [&](int nt) {
            if constexpr (NORM) {
                const int col = 16 * nt + j16;
                return sS[(g & 3) * EB + (col < C::NCOLS ? col / NORB : 0)];
            } else {
                return 1.0;
            }
        };
#pragma unroll
        for (int nt = 0; nt < C::NT; ++nt) {
            const double f = inv_of(nt);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[nt][v] = NORM ? fma((double)part[nt][v], f, acc[nt][v]) : acc[nt][v] + (double)part[nt][v];
        }
        const double fx = inv_of(ext_nt);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc_x[v] = NORM ? fma((double)part_x[v], fx, acc_x[v]) : acc_x[v] + (double)part_x[v];
    };

    // ---- add one V tile of energy block blk into the output ring
    // Source energy es feeds Sigma at es + w through the terms with G at E - w
    // and Sigma at es - w through those with G at E + w; FLAGS keeps either set.
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
            const int row = 16 * mt + 4 * kk + v;  // fp32 accumulator layout of the 16x16 tiles
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

    // ---- every wave runs the phases in the same order: the P tiles of the next
    // chunk, the X rows of the chunk after (from G loads issued at the end of the
    // previous chunk), the main GEMM of this chunk at a raised issue priority
    // (its matrix instructions then start as soon as their operands are in,
    // and the vector work of the other wave on the SIMD fills the gaps), and the
    // G gather of a later chunk, in flight across the barrier and the next P
    // tiles.  Every phase has one call site, which keeps the accumulators in
    // place across the loop.  (Measured at the device workload against the two
    // waves of a SIMD running opposite orders: 838 -> 752 ms for fp16 hi/lo.)

    // ---- prologue: X for chunks 0 and 1, P for chunk 0, G for chunk 2
    __syncthreads();
    gather_g(0);
    finish_x(0);
    __syncthreads();
    gather_g(1);
    p_tiles(0);
    finish_x(1);
    gather_g(2);
    __syncthreads();

    // ---- main loop: energy blocks, one K chunk per momentum k', one barrier per chunk
    for (int blk = 0; blk < nblk; ++blk) {
#pragma unroll
        for (int nt = 0; nt < C::NT; ++nt) acc[nt] = f64x4{0.0, 0.0, 0.0, 0.0};
        acc_x = f64x4{0.0, 0.0, 0.0, 0.0};
        for (int ch = 0; ch < NKZ; ++ch) {
            const int g = blk * NKZ + ch;
            p_tiles(g + 1);
            finish_x(g + 2);  // G for chunk g+2 was gathered at the end of chunk g-1
            __builtin_amdgcn_s_setprio(1);
            mfma_chunk(g);
            __builtin_amdgcn_s_setprio(0);
            gather_g(g + 3);
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

template <int NORB, int NKZ, int NW, int NB, int PREC, int FLAGS>
static hipError_t launch_h16_flags(const Dims& d, const double* G, const double* D, const double* A,
                                   const double* B, const int32_t* nbr, cd alpha, double* S, hipStream_t stream) {
    constexpr int EB = 8;
    using C = H16Cfg<NORB, NKZ, NW, NB, EB>;
    auto kern = fwd_h16_kernel<NORB, NKZ, NW, NB, EB, PREC, FLAGS>;
    // set on every launch (cheap): the attribute is per device, and a process-wide
    // flag would race between host threads
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)C::LDS_BYTES);
    if (e != hipSuccess) return e;
    const int64_t groups = ((d.na + 7) / 8) * 8 * NORB;
    hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(C::THREADS), C::LDS_BYTES, stream, d, G, D, A, B, nbr, alpha,
                       S);
    return hipGetLastError();
}

template <int NORB, int NKZ, int NW, int NB, int PREC>
static hipError_t launch_h16(const Dims& d, const double* G, const double* D, const double* A, const double* B,
                             const int32_t* nbr, cd alpha, double* S, hipStream_t stream, int flags) {
    constexpr int kBoth = kBranchMinus | kBranchPlus, kPlusAdd = kBranchPlus | kAccumulate;
    if (flags == kBoth) return launch_h16_flags<NORB, NKZ, NW, NB, PREC, kBoth>(d, G, D, A, B, nbr, alpha, S, stream);
    if constexpr (Split16<PREC>::LO) {  // the single-term forms take one table only
        if (flags == kBranchMinus)
            return launch_h16_flags<NORB, NKZ, NW, NB, PREC, kBranchMinus>(d, G, D, A, B, nbr, alpha, S, stream);
        if (flags == kPlusAdd)
            return launch_h16_flags<NORB, NKZ, NW, NB, PREC, kPlusAdd>(d, G, D, A, B, nbr, alpha, S, stream);
    }
    return hipErrorInvalidValue;
}

template <int PREC>
static hipError_t dispatch_h16(const Dims& d, const double* G, const double* D, const double* A, const double* B,
                               const int32_t* nbr, cd alpha, double* S, hipStream_t stream, int flags) {
    if (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 4)
        return launch_h16<10, 7, 10, 4, PREC>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (d.norb == 10 && d.nkz == 7 && d.nw == 10 && d.nb == 3)
        return launch_h16<10, 7, 10, 3, PREC>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (d.norb == 4 && d.nkz == 3 && d.nw == 2 && d.nb == 4)
        return launch_h16<4, 3, 2, 4, PREC>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    return hipErrorInvalidValue;
}

hipError_t launch_fwd_h16(const Dims& d, int precision, const double* G, const double* D, const double* A,
                          const double* B, const int32_t* nbr, cd alpha, double* S, hipStream_t stream, int flags) {
    if (precision == SSE_FP16X2) return dispatch_h16<SSE_FP16X2>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (precision == SSE_BF16X2) return dispatch_h16<SSE_BF16X2>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (precision == SSE_FP16) return dispatch_h16<SSE_FP16>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    if (precision == SSE_FP16_UNSCALED)
        return dispatch_h16<SSE_FP16_UNSCALED>(d, G, D, A, B, nbr, alpha, S, stream, flags);
    return hipErrorInvalidValue;
}

}  // namespace sse
