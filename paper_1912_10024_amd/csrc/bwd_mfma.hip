// Matrix-core adjoint of the scattering self-energy (Eq. 3): dG and d gradH in fp64.
//
// With g = dL/dSigma (PyTorch's complex-gradient convention) and, for an edge
// (a, n) with neighbour b = nbr[a,n] and A_i = grad_i H_{a,n},
//   W[k,w,E']   = g[k, E'+w, a] + g[k, E'-w, a]                    (0 outside the energy grid)
//   Y_ij[k',E'] = sum_{q,w} Dc_ij[q,w] W[(k'+q) mod Nkz, w, E'],   Dc = conj(alpha D[q,w-1,a,n,i,j])
// the gradients with respect to G and grad H are
//   dG[k',E',b,0] = sum over the edges into b of  sum_j T_j A_j,    T_m = sum_i A_i^H Y_im
//   dA_m          = sum_{k',E'} U_m B^H + T_m^H B,                  U_m = sum_j Y_mj A_j
// with B = G[k',E',b,0] (the adjoint of the stencil, of the D contraction and
// of P = A_i B A_j^H).
//
// Y is the forward's dense contraction transposed.  For a pair of energies E':
//   Y^T[(E', r, c)][(k', i, j)] = sum_{(k, w)} W[k, w, E'][r][c] * Dc[(k - k') mod Nkz, w, i, j]
// a GEMM with 2 Norb^2 rows, K = Nkz Nw complex and Nkz * 9 complex columns;
// the momentum convolution is the circulant structure of the coefficient
// operand.  It runs on v_mfma_f64_16x16x4_f64, the real embedding of the
// complex product on the coefficient side ([[Re, Im], [-Im, Re]] per entry,
// a static LDS table), W formed per momentum k from g in global memory and
// staged in LDS.  The small products (U, T^H, the dG term and the d gradH
// terms) run one momentum k' at a time as batched GEMMs on the same matrix
// instruction: their left operands are read from LDS copies of Y, U and T^H,
// their right operands from embedded tables of A (per edge) and of B and
// conj(B)^T (per momentum and energy pair).
//
// Work decomposition: one workgroup of 8 waves per (neighbour atom b, range
// of 32 energies) walks the edges into b in edge order (the reverse
// adjacency).  Every dG element has one owner: the first edge writes it, the
// later ones add to it in edge order.  d gradH of an edge gets one partial sum
// per energy range, added in range order by the reduce kernel.  No atomics:
// bitwise reproducible.  A workgroup's time grows with the in-degree of b
// (Poisson-like for a random neighbour table), so the workgroups are
// dispatched in decreasing in-degree (the order array): the long ones start
// first instead of leaving a tail of idle compute units.  The order changes no
// result.
#include "sse_kernels.h"

namespace sse {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mma(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ double neg_if(double x, bool neg) {
    return __longlong_as_double(__double_as_longlong(x) ^ (neg ? (long long)0x8000000000000000ull : 0ll));
}

// A chain of NS dependent matrix instructions on one accumulator, its operands
// read (LDS) up front in step order; the scheduler interleaves the reads with
// the chain as registers allow.
template <int NS, class FA, class FB>
__device__ __forceinline__ f64x4 mma_chain(FA fa, FB fb, f64x4 c) {
    double a[NS], b[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        a[s] = fa(s);
        b[s] = fb(s);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) c = mma(a[s], b[s], c);
    return c;
}

}  // namespace

template <int NORB, int NKZ, int NW, int EP_>
struct BwdCfg {
    static constexpr int WAVES = 8, THREADS = 64 * WAVES;
    static constexpr int NN = NORB * NORB;
    static constexpr int EP = EP_;  // energies per main-GEMM step
    static constexpr int ECH = 32;  // energies per workgroup
    // main GEMM: rows (ep, r, c), K per momentum k = (w, re/im), columns (k', i, j, re/im)
    static constexpr int MROWS = EP * NN;
    static constexpr int MT = (MROWS + 15) / 16;
    static constexpr int MPAD = MT * 16;
    static constexpr int KC = 2 * NW;
    static constexpr int KS = KC / 4;
    static constexpr int NCOL = NKZ * 18;
    static constexpr int NT = (NCOL + 15) / 16;
    // small products: K rows (j, c, re/im) per block j, table width (c', re/im) padded
    static constexpr int K2 = 2 * NORB;
    static constexpr int KA = 3 * K2;
    static constexpr int TW = 40;  // row stride of the tables: the four rows of an operand read use
                                   // the two halves of the banks
    static constexpr int PR = EP * 3 * NORB;  // rows (ep, m, r) of U and T^H
    static constexpr int GR = EP * NORB;      // rows (ep, x) of the dG term
    static constexpr int AR = 3 * NORB;       // rows (m, r) of d gradH
    static constexpr int KB = 2 * EP * K2;    // K rows of the d gradH terms (U half, T^H half)
    // LDS (doubles)
    static constexpr int L_W = KC * MPAD;          // W of one momentum [w, re/im][ep, r, c] (two buffers)
    static constexpr int L_DC = NKZ * NW * 9 * 4;  // embedded Dc [q][w][ij][4]
    // Y of one momentum [ep][ij][r][c] complex, YB doubles per (ep, ij) block: the
    // padding spreads the rows (m, r) of an operand read over the banks
    static constexpr int YB = 2 * NN + 12;
    static constexpr int L_Y = EP * 9 * YB;  // (two buffers)
    static constexpr int L_U = EP * 3 * NN * 2;    // U and T^H [ep][m][r][c] complex (two buffers each)
    static constexpr int L_TA = KA * TW;           // embedded A [j, c, re/im][c', re/im]
    static constexpr int L_TB = KB * TW;           // embedded conj(B)^T and B (two buffers)
    static constexpr size_t LDS_BYTES = 8 * (size_t)(2 * L_W + L_DC + 2 * L_Y + 4 * L_U + L_TA + 2 * L_TB);
    static_assert(NT == WAVES, "one column tile of the main GEMM per wave");
    static_assert(KC % 4 == 0 && K2 % 4 == 0, "a K step never straddles a frequency pair or a block j");
    static_assert(K2 <= TW, "table width");
    static constexpr int NPAIR = (PR + 15) / 16 * 2;  // (row tile, column tile) pairs of U and T^H
    static_assert((K2 + 15) / 16 == 2, "two column tiles in the small products");
    static_assert(NPAIR == 8 || NPAIR == 4, "U and T^H: both products of one pair per wave, or one of them");
    static_assert(GR <= 16 && (AR + 15) / 16 == 2, "dG term: two tiles (waves 2, 3); d gradH: four (waves 0, 1, 4, 5)");
    static_assert(NN % 4 == 0, "the four rows of an output lane group share one energy");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
};

template <int NORB, int NKZ, int NW, int EP>
__global__ __launch_bounds__(512) void bwd_mfma_kernel(Dims d, const double* __restrict__ G,
                                                       const double* __restrict__ Dg, const double* __restrict__ Ag,
                                                       const double* __restrict__ gS, cd calpha,
                                                       const int32_t* __restrict__ offset,
                                                       const int32_t* __restrict__ edges,
                                                       const int32_t* __restrict__ order, double* __restrict__ dG,
                                                       double* __restrict__ dApart) {
    using C = BwdCfg<NORB, NKZ, NW, EP>;
    constexpr int NN = C::NN, K2 = C::K2, TW = C::TW, MPAD = C::MPAD;
    extern __shared__ double lds[];
    double* sW = lds;
    double* sDc = sW + 2 * C::L_W;
    double* sY = sDc + C::L_DC;
    double* sU = sY + 2 * C::L_Y;
    double* sT = sU + 2 * C::L_U;
    double* sTA = sT + 2 * C::L_U;
    double* sTB = sTA + C::L_TA;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l4 = lane >> 4, l16 = lane & 15;
    // energies fit 32 bits: the dispatcher admits ne < 2^28
    const int NE = (int)d.ne;
    const int nch = (NE + C::ECH - 1) / C::ECH;
    // atoms in decreasing in-degree: the longest workgroups are dispatched first
    if (blockIdx.x / nch >= d.na) return;  // uniform for the workgroup, before any barrier
    const int64_t b = order[blockIdx.x / nch];
    const int ch = (int)(blockIdx.x % nch);
    const int E_lo = ch * C::ECH, E_hi = E_lo + C::ECH < NE ? E_lo + C::ECH : NE;
    const int32_t e_lo = offset[b], e_hi = offset[b + 1];

    // slots >= 1 of dG are not read by the forward map: zero; with no edge into
    // b, slot 0 of this energy range is zero too
    if (dG && (d.gs > 1 || e_lo == e_hi)) {
        const int from = e_lo == e_hi ? 0 : NN;
        for (int k = 0; k < NKZ; ++k)
            for (int E = E_lo; E < E_hi; ++E) {
                const int64_t base = off_G(d, k, E, b);
                for (int64_t x = from + tid; x < d.gs * NN; x += C::THREADS) cstore(dG, base + x, cd{0.0, 0.0});
            }
    }
    if (e_lo == e_hi) return;  // uniform

    // main GEMM, this wave's column tile: (k', ij, re/im) of the lane's column
    const int col = 16 * wave + l16;
    const int kpc = col < C::NCOL ? col / 18 : 0;  // padding columns: any in-bounds entry
    const int ijc = (col % 18) >> 1, ccc = col & 1;
    // B fragment of K step s: row 4 s + l4 = (w = 2 s + l4 / 2, re/im = l4 & 1)
    const int dc_lane = ((l4 >> 1) * 9 + ijc) * 4 + 2 * (l4 & 1) + ccc;
    const double* pa_main = sW + l4 * MPAD + l16;

    // W items of this thread: (w, ep, r c) = tid + THREADS u
    constexpr int NITEM = NW * C::EP * NN;
    constexpr int NU = (NITEM + C::THREADS - 1) / C::THREADS;
    // B items of this thread: (k', ep, p q) = tid + THREADS u
    constexpr int NBITEM = NKZ * C::EP * NN;
    constexpr int NUB = (NBITEM + C::THREADS - 1) / C::THREADS;

    f64x4 dacc = {0.0, 0.0, 0.0, 0.0};  // d gradH tile of waves 4..7, per edge
    for (int32_t ei = e_lo; ei < e_hi; ++ei) {
        const int32_t edge = edges[ei];
        const int64_t a = edge / d.nb, n = edge % d.nb;
        __syncthreads();  // the previous edge's readers of the tables are done
        // Dc = conj(alpha D) = conj(alpha) conj(D), embedded as (Re, Im, -Im, Re)
        for (int x = tid; x < NKZ * NW * 9; x += C::THREADS) {
            const int ij = x % 9, w = (x / 9) % NW, q = x / (9 * NW);
            const cd v = cload(Dg, off_D(d, q, w, a, n) + ij);
            const cd z = cmul(calpha, cd{v.re, -v.im});
            double* o = sDc + 4 * x;
            o[0] = z.re;
            o[1] = z.im;
            o[2] = -z.im;
            o[3] = z.re;
        }
        // A_j[c][c'] at row (j, c, re/im), column (c', re/im)
        for (int x = tid; x < 3 * NN; x += C::THREADS) {
            const int j = x / NN, c = (x % NN) / NORB, cp = x % NORB;
            const cd v = cload(Ag, off_A(d, a, n, j) + c * NORB + cp);
            double* o = sTA + (j * K2 + 2 * c) * TW + 2 * cp;
            o[0] = v.re;
            o[1] = v.im;
            o[TW] = -v.im;
            o[TW + 1] = v.re;
        }
        dacc = f64x4{0.0, 0.0, 0.0, 0.0};
        const double* gA = gS + 2 * off_S(d, 0, 0, a);  // g of atom a at (k, E) = 0
        // dG entries of this lane in the dG-term waves (rows (ep, x), columns (u, re/im)):
        // the first edge writes them, later edges add to the previous edge's
        // values, read one round ahead
        const int64_t g_k = 2 * d.ne * d.na * d.gs * NN;  // one momentum further in dG
        int64_t g_off[4];
        bool g_ok[4];
        double gprev[4];
        auto set_prev = [&](int E0) {
            const int cl = 16 * (wave - 2) + l16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int orow = 4 * v + l4, o_ep = orow / NORB, o_x = orow % NORB;
                g_ok[v] = orow < C::GR && cl < K2 && E0 + o_ep < NE;
                g_off[v] = 2 * (off_G(d, 0, g_ok[v] ? E0 + o_ep : 0, b) + o_x * NORB) + cl;
            }
        };
        auto load_prev = [&](int kp, double* dst) {
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[v] = (ei != e_lo && g_ok[v]) ? dG[g_off[v] + g_k * kp] : 0.0;
        };
        const int64_t stride_e = 2 * d.na * NN, stride_k = stride_e * d.ne;

        // W items of this thread for the energies from E0: offsets of the two shifted blocks
        int64_t rel_p[NU], rel_m[NU];
        bool ok_p[NU], ok_m[NU];
        auto set_items = [&](int E0) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int i = tid + C::THREADS * u;
                const int rc = i % NN, ep = (i / NN) % C::EP, w = i / (NN * C::EP) + 1;
                const int E = E0 + ep;
                const bool in = i < NITEM && E < NE;  // i >= NITEM: w beyond NW, never in
                ok_p[u] = in && E + w < NE;
                ok_m[u] = in && E - w >= 0;
                // energies outside the grid read energy 0 of the atom (in bounds) and count as zero
                rel_p[u] = (int64_t)(ok_p[u] ? E + w : 0) * stride_e + 2 * rc;
                rel_m[u] = (int64_t)(ok_m[u] ? E - w : 0) * stride_e + 2 * rc;
            }
        };
        cd gp[NU], gm[NU];
        auto gather = [&](int k) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const double2 vp = *reinterpret_cast<const double2*>(gA + k * stride_k + rel_p[u]);
                const double2 vm = *reinterpret_cast<const double2*>(gA + k * stride_k + rel_m[u]);
                gp[u] = ok_p[u] ? cd{vp.x, vp.y} : cd{0.0, 0.0};
                gm[u] = ok_m[u] ? cd{vm.x, vm.y} : cd{0.0, 0.0};
            }
        };
        auto store_w = [&](int buf) {
            double* w = sW + buf * C::L_W;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int i = tid + C::THREADS * u;
                if (i < NITEM) {
                    const int row = i % (NN * C::EP), wi = i / (NN * C::EP);
                    w[(2 * wi) * MPAD + row] = gp[u].re + gm[u].re;
                    w[(2 * wi + 1) * MPAD + row] = gp[u].im + gm[u].im;
                }
            }
        };
        // the first momentum of the first energies; later ones are stored in
        // the product rounds of the energies before
        set_items(E_lo);
        gather(0);
        store_w(0);
        __syncthreads();

        for (int E0 = E_lo; E0 < E_hi; E0 += C::EP) {
            // the neighbour's G blocks of every momentum at these energies, read
            // during the GEMM and staged as tables in the product rounds
            cd bpre[NUB];
#pragma unroll
            for (int u = 0; u < NUB; ++u) {
                const int x = tid + C::THREADS * u;
                const int kp = x / (C::EP * NN), ep = (x / NN) % C::EP, pq = x % NN;
                bpre[u] = cd{0.0, 0.0};
                if (x < NBITEM && E0 + ep < NE) bpre[u] = cload(G, off_G(d, kp, E0 + ep, b) + pq);
            }

            // the previous edge's dG of the first momentum (added to in the first round)
            if (dG && (wave == 2 || wave == 3)) {
                set_prev(E0);
                load_prev(0, gprev);
            }

            f64x4 acc[C::MT];
#pragma unroll
            for (int mt = 0; mt < C::MT; ++mt) acc[mt] = f64x4{0.0, 0.0, 0.0, 0.0};
            // momentum k in buffer k & 1: it is written while the other buffer is
            // read, and the barrier that ends momentum k - 1 orders the two
            for (int k = 0; k < NKZ; ++k) {
                if (k + 1 < NKZ) gather(k + 1);
                int q = k - kpc;
                if (q < 0) q += NKZ;
                const double* pb = sDc + q * NW * 36 + dc_lane;
                const double* pa = pa_main + (k & 1) * C::L_W;
                // operands of K step s + 1 are read while the instructions of step s run
                double an[C::MT], bn = pb[0];
#pragma unroll
                for (int mt = 0; mt < C::MT; ++mt) an[mt] = pa[16 * mt];
#pragma unroll
                for (int s = 0; s < C::KS; ++s) {
                    double ac[C::MT];
#pragma unroll
                    for (int mt = 0; mt < C::MT; ++mt) ac[mt] = an[mt];
                    const double bc = bn;
                    if (s + 1 < C::KS) {
#pragma unroll
                        for (int mt = 0; mt < C::MT; ++mt) an[mt] = pa[4 * (s + 1) * MPAD + 16 * mt];
                        bn = pb[72 * (s + 1)];
                    }
#pragma unroll
                    for (int mt = 0; mt < C::MT; ++mt) acc[mt] = mma(ac[mt], bc, acc[mt]);
                }
                if (k + 1 < NKZ) store_w((k + 1) & 1);
                __syncthreads();
            }
            // the first momentum of the next energies, read during the product rounds
            if (E0 + C::EP < E_hi) {
                set_items(E0 + C::EP);
                gather(0);
            }

            // ---- the small products, pipelined over the momenta k'.  Phase kp runs U
            // and T^H of kp (sY buffer kp & 1 into sU / sT buffer kp & 1), the dG and
            // d gradH terms of kp - 1 (sU / sT and table buffer (kp - 1) & 1), and
            // stages Y of kp + 1 and the B tables of kp; one barrier per phase.  Every
            // buffer a phase writes was last read two phases earlier.
            auto stage_y = [&](int kp) {
                // Y of momentum kp from the columns that carry it
                // (row 16 mt + 4 v + l4 lies in energy (16 mt + 4 v) / NN: NN is a multiple of 4)
                if (kpc == kp && col < C::NCOL) {
                    double* py = sY + (kp & 1) * C::L_Y + ijc * C::YB + ccc + 2 * l4;
#pragma unroll
                    for (int mt = 0; mt < C::MT; ++mt)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int r0 = 16 * mt + 4 * v;
                            if (r0 < C::MROWS) {
                                const int ep = r0 / NN;
                                py[ep * 9 * C::YB + (r0 - ep * NN) * 2] = acc[mt][v];
                            }
                        }
                }
            };
            auto stage_tb = [&](int kp) {
                // conj(B)^T at rows (ep, c', re/im), columns (c, re/im); B at rows
                // KB/2 + (ep, q, re/im), columns (c, re/im)
                double* tb = sTB + (kp & 1) * C::L_TB;
#pragma unroll
                for (int u = 0; u < NUB; ++u) {
                    const int x = tid + C::THREADS * u;
                    if (x < NBITEM && x / (C::EP * NN) == kp) {
                        const int ep = (x / NN) % C::EP, p = (x % NN) / NORB, qq = x % NORB;
                        const cd v = bpre[u];
                        double* o1 = tb + (ep * K2 + 2 * qq) * TW + 2 * p;
                        o1[0] = v.re;
                        o1[1] = -v.im;
                        o1[TW] = v.im;
                        o1[TW + 1] = v.re;
                        double* o2 = tb + (C::EP * K2 + ep * K2 + 2 * p) * TW + 2 * qq;
                        o2[0] = v.re;
                        o2[1] = v.im;
                        o2[TW] = -v.im;
                        o2[TW + 1] = v.re;
                    }
                }
            };
            // U_m[ep][r][c'] = sum_{j,c} Y_mj[r][c] A_j[c][c'] and
            // T^H_m[ep][p][q] = sum_{i,r} conj(Y_im[r][p]) A_i[r][q]: rows (ep, m, r)
            auto uv = [&](int kp) {
                const double* yb = sY + (kp & 1) * C::L_Y;
                double* ub = sU + (kp & 1) * C::L_U;
                double* tb = sT + (kp & 1) * C::L_U;
                const int pair = C::NPAIR == 8 ? wave : (wave & 3);
                const bool do_u = C::NPAIR == 8 || wave < 4, do_t = C::NPAIR == 8 || wave >= 4;
                const int mt = pair >> 1, nt = pair & 1;
                int row = 16 * mt + l16;
                if (row >= C::PR) row = C::PR - 1;  // padding rows: any in-bounds row
                const int ep = row / (3 * NORB), m = (row / NORB) % 3, r = row % NORB;
                const double* pa1 = yb + (ep * 9 + m * 3) * C::YB + r * NORB * 2 + l4;
                const double* pa2 = yb + (ep * 9 + m) * C::YB + 2 * r + (l4 >> 1) * 2 * NORB + (l4 & 1);
                const double* pb = sTA + l4 * TW + 16 * nt + l16;
                const bool neg = (l4 & 1) != 0;
                const int cl = 16 * nt + l16;
                // one straight-line product per path (the choice is uniform per wave)
                auto store_tile = [&](double* dst, const f64x4& c) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int orow = 16 * mt + 4 * v + l4;
                        if (orow < C::PR && cl < K2) {
                            const int o_ep = orow / (3 * NORB), o_m = (orow / NORB) % 3, o_r = orow % NORB;
                            dst[((o_ep * 3 + o_m) * NN + o_r * NORB) * 2 + cl] = c[v];
                        }
                    }
                };
                const f64x4 zero = {0.0, 0.0, 0.0, 0.0};
                auto b_of = [&](int s) { return pb[4 * s * TW]; };
                if (do_u) {
                    const f64x4 cu = mma_chain<C::KA / 4>(
                        [&](int s) { return pa1[(4 * s / K2) * C::YB + (4 * s) % K2]; }, b_of, zero);
                    store_tile(ub, cu);
                }
                if (do_t) {
                    const f64x4 ct = mma_chain<C::KA / 4>(
                        [&](int s) { return neg_if(pa2[(4 * s / K2) * 3 * C::YB + ((4 * s) % K2) * NORB], neg); },
                        b_of, zero);
                    store_tile(tb, ct);
                }
            };
            auto terms = [&](int kp) {
                const double* ub = sU + (kp & 1) * C::L_U;
                const double* tb = sT + (kp & 1) * C::L_U;
                if (wave == 2 || wave == 3) {
                    // dG[ep][x][u] (+)= sum_{j,c} conj(T^H_j[ep][c][x]) A_j[c][u]: rows (ep, x)
                    if (dG) {
                        const int nt = wave - 2;
                        int row = l16;
                        if (row >= C::GR) row = C::GR - 1;
                        const int ep = row / NORB, x = row % NORB;
                        const double* pa = tb + (ep * 3 * NN + x) * 2 + (l4 >> 1) * 2 * NORB + (l4 & 1);
                        const double* pb = sTA + l4 * TW + 16 * nt + l16;
                        const bool neg = (l4 & 1) != 0;
                        // the next momentum's previous values are read before this
                        // momentum's stores are issued: a wait for those loads then
                        // does not also wait for the stores
                        double gnext[4] = {0.0, 0.0, 0.0, 0.0};
                        if (kp + 1 < NKZ) load_prev(kp + 1, gnext);
                        const f64x4 cg = mma_chain<C::KA / 4>(
                            [&](int s) { return neg_if(pa[(4 * s / K2) * 2 * NN + ((4 * s) % K2) * NORB], neg); },
                            [&](int s) { return pb[4 * s * TW]; }, f64x4{0.0, 0.0, 0.0, 0.0});
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            if (g_ok[v]) dG[g_off[v] + g_k * kp] = gprev[v] + cg[v];
                            gprev[v] = gnext[v];
                        }
                    }
                } else if (dApart && wave < 6) {
                    // dA_m[r][c] += sum_{ep,c'} U_m[ep][r][c'] conj(B_ep[c][c'])
                    //             + sum_{ep,q} T^H_m[ep][r][q] B_ep[q][c]: rows (m, r);
                    // waves 0, 1, 4, 5, so that each SIMD carries at most two of the
                    // four tiles of this product
                    const int w4 = (wave & 1) + 2 * (wave >> 2), mt = w4 >> 1, nt = w4 & 1;
                    int row = 16 * mt + l16;
                    if (row >= C::AR) row = C::AR - 1;
                    const int m = row / NORB, r = row % NORB;
                    const int arow = (m * NN + r * NORB) * 2 + l4;
                    const double* pb = sTB + (kp & 1) * C::L_TB + l4 * TW + 16 * nt + l16;
                    dacc = mma_chain<C::KB / 4>(
                        [&](int s) {
                            const int t0 = 4 * s, th = t0 % (C::EP * K2);
                            return (t0 / (C::EP * K2) ? tb : ub)[arow + (th / K2) * 6 * NN + th % K2];
                        },
                        [&](int s) { return pb[4 * s * TW]; }, dacc);
                }
            };
            stage_y(0);
            __syncthreads();
            for (int kp = 0; kp <= NKZ; ++kp) {
                if (kp < NKZ) uv(kp);
                if (kp > 0) terms(kp - 1);
                if (kp + 1 < NKZ) stage_y(kp + 1);
                if (kp < NKZ) stage_tb(kp);
                // the first W of the next energies (buffer 0, last read by the GEMM's
                // final momentum)
                if (kp == NKZ && E0 + C::EP < E_hi) store_w(0);
                __syncthreads();
            }
        }
        // this energy range's share of the edge's d gradH
        if (dApart && (wave < 2 || wave == 4 || wave == 5)) {
            const int w4 = (wave & 1) + 2 * (wave >> 2), mt = w4 >> 1, nt = w4 & 1;
            const int cl = 16 * nt + l16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int orow = 16 * mt + 4 * v + l4;
                if (orow < C::AR && cl < K2) {
                    const int m = orow / NORB, r = orow % NORB;
                    dApart[2 * (((int64_t)ch * d.na * d.nb + edge) * 3 * NN + m * NN + r * NORB) + cl] = dacc[v];
                }
            }
        }
    }
}

// energies per main-GEMM step: 1 keeps the accumulators of a wave at 56 registers
constexpr int kBwdEP = 1;
using BwdC = BwdCfg<10, 7, 10, kBwdEP>;

bool bwd_mfma_specialised(const Dims& d) { return d.norb == 10 && d.nkz == 7 && d.nqz == 7 && d.nw == 10; }

int64_t bwd_mfma_shares(const Dims& d) { return (d.ne + BwdC::ECH - 1) / BwdC::ECH; }

hipError_t bwd_mfma_prepare() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(bwd_mfma_kernel<10, 7, 10, kBwdEP>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)BwdC::LDS_BYTES);
}

hipError_t launch_bwd_mfma(const Dims& d, const double* G, const double* D, const double* A, const double* gS, cd calpha,
                           const int32_t* offset, const int32_t* edges, const int32_t* order, double* dG,
                           double* dApart, hipStream_t stream) {
    const int64_t groups = d.na * bwd_mfma_shares(d);
    hipLaunchKernelGGL((bwd_mfma_kernel<10, 7, 10, kBwdEP>), dim3((unsigned)groups), dim3(BwdC::THREADS),
                       BwdC::LDS_BYTES, stream, d, G, D, A, gS, calpha, offset, edges, order, dG, dApart);
    return hipGetLastError();
}

}  // namespace sse
