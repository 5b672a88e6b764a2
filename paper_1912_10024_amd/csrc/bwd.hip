// Adjoint of the scattering self-energy (fp64, vector ALUs).
//
// With g = dL/dSigma (PyTorch's complex-gradient convention) define, for an
// edge (a, n) with neighbour b = nbr[a,n] and a source point (k', E'):
//   W_{q,w}[k',E'] = g[(k'+q) mod Nkz, E'+w, a] + g[(k'+q) mod Nkz, E'-w, a]   (0 outside the grid)
//   Y_ij[k',E']    = conj(alpha) sum_{q,w} conj(D[q,w-1,a,n,i,j]) W_{q,w}[k',E']
// (the adjoint of the (qz, w, +/-) stencil and of the D contraction; over
// signed frequencies the g at E'+w term takes conj(Dp) and the one at E'-w
// conj(Dm)), and with
// B = G[k',E',b,0], P_ij = grad_i H . B . grad_j H^H:
//   dG[k',E',b,0]   += sum_ij grad_i H^H . Y_ij . grad_j H
//   d gradH[a,n,m]  += sum_j Y_mj . (grad_j H . B^H) + sum_i Y_im^H . (grad_i H . B)
//   dD[q,w-1,a,n,ij] = conj(alpha) sum_{k',E'} sum_rc conj(P_ij[rc]) W_{q,w}[rc]
//   (over signed frequencies: dDp from the g at E'+w terms, dDm from E'-w)
// Shifted blocks are re-gathered from G and g, nothing of the forward is stored.
//
// dG and d gradH are formed by one workgroup per neighbour atom b, which walks
// the edges that point at b (a reverse adjacency built in the workspace, in
// edge order), so every output element has one owner: no atomics, bitwise
// reproducible.  dD is formed by one workgroup per edge here, or by the
// matrix-core phonon kernel in its adjoint mode for the shape it covers.
#include <algorithm>

#include "sse_kernels.h"

namespace sse {

namespace {
constexpr int kBwdThreads = 256;
constexpr int kYHalf = kBwdThreads / 2;   // first thread of the second Y group
}

// ---------------------------------------------------------------- reverse adjacency
// ws layout (int32): count[na] | offset[na+1] | cursor[na] | edges[na*nb]
__global__ void rcsr_count_kernel(int64_t na, int64_t nb, const int32_t* __restrict__ nbr, int32_t* count) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < na * nb; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = nbr[x];
        if (b >= 0 && b < na) atomicAdd(&count[b], 1);
    }
}

// single workgroup exclusive scan (na is at most a few hundred thousand)
__global__ void rcsr_scan_kernel(int64_t na, const int32_t* __restrict__ count, int32_t* offset, int32_t* cursor) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t per = (na + nt - 1) / nt;
    const int64_t lo = tid * per, hi = (lo + per < na) ? lo + per : na;
    int32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += count[i];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int t = 0; t < nt; ++t) {
            const int32_t v = part[t];
            part[t] = run;
            run += v;
        }
        offset[na] = run;
    }
    __syncthreads();
    int32_t run = part[tid];
    for (int64_t i = lo; i < hi; ++i) {
        offset[i] = run;
        cursor[i] = run;
        run += count[i];
    }
}

__global__ void rcsr_fill_kernel(int64_t na, int64_t nb, const int32_t* __restrict__ nbr, int32_t* cursor, int32_t* edges) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < na * nb; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = nbr[x];
        if (b >= 0 && b < na) edges[atomicAdd(&cursor[b], 1)] = (int32_t)x;
    }
}

// the fill order is arbitrary: sort each (short) list so the walk is in edge order
__global__ void rcsr_sort_kernel(int64_t na, const int32_t* __restrict__ offset, int32_t* edges) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < na; b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t lo = offset[b], hi = offset[b + 1];
        for (int32_t i = lo + 1; i < hi; ++i) {
            const int32_t v = edges[i];
            int32_t j = i - 1;
            while (j >= lo && edges[j] > v) {
                edges[j + 1] = edges[j];
                --j;
            }
            edges[j + 1] = v;
        }
    }
}

// atoms in decreasing in-degree (the dispatch order of both dG / d gradH kernels:
// a workgroup's time grows with the in-degree of its atom, so the longest start
// first and the shortest fill the end).  One workgroup; degrees above 255
// share the first bucket; the order within a bucket is arbitrary, which changes
// no result (every workgroup of that kernel owns its outputs).
__global__ __launch_bounds__(1024) void rcsr_order_kernel(int64_t na, const int32_t* __restrict__ count,
                                                          int32_t* __restrict__ order) {
    __shared__ int32_t cursor[256];
    const int tid = threadIdx.x;
    if (tid < 256) cursor[tid] = 0;
    __syncthreads();
    auto bucket = [&](int64_t a) { return 255 - (count[a] < 255 ? count[a] : 255); };
    for (int64_t a = tid; a < na; a += 1024) atomicAdd(&cursor[bucket(a)], 1);
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int k = 0; k < 256; ++k) {
            const int32_t c = cursor[k];
            cursor[k] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int64_t a = tid; a < na; a += 1024) order[atomicAdd(&cursor[bucket(a)], 1)] = (int32_t)a;
}

__global__ void zero_i32_kernel(int64_t n, int32_t* p) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) p[x] = 0;
}

// ws layout after the reverse adjacency (256-byte aligned): the d gradH sums of
// every edge, one set per momentum k' (complex [nkz][na*nb][3][norb][norb]),
// added in k' order by bwd_dh_reduce_kernel (one per range of energies on the
// matrix cores), if d gradH is asked for; then the atom-major copy of g that
// the matrix-core D gradient reads, if dD is asked for with copy_g
static size_t bwd_csr_bytes(const Dims& d) {  // count, offset, cursor, edges, order
    return (sizeof(int32_t) * (size_t)(4 * d.na + 1 + d.na * d.nb) + 255) / 256 * 256;
}
// the matrix-core kernel keeps one d gradH share per range of energies instead
static bool bwd_use_mfma(const Dims& d, bool signed_form) {
    return !signed_form && bwd_mfma_specialised(d) && d.ne < (int64_t(1) << 28) &&
           d.na * bwd_mfma_shares(d) <= INT32_MAX;
}
static int64_t bwd_shares(const Dims& d, bool signed_form) {
    return bwd_use_mfma(d, signed_form) ? bwd_mfma_shares(d) : d.nkz;
}
static size_t bwd_dh_bytes(const Dims& d, bool signed_form) {
    return (sizeof(cd) * (size_t)(bwd_shares(d, signed_form) * d.na * d.nb * 3 * d.norb * d.norb) + 255) / 256 * 256;
}
size_t bwd_workspace_bytes_for(const Dims& d, bool signed_form, bool with_dh, bool with_dd, bool copy_g) {
    // only the one-table form reads both energy branches of g per GEMM row, whose
    // window is the one that the atom-major copy keeps within a few pages
    return bwd_csr_bytes(d) + (with_dh ? bwd_dh_bytes(d, signed_form) : 0) +
           (with_dd && copy_g && !signed_form ? pse_atom_major_bytes(d) : 0);
}
size_t bwd_workspace_bytes(const Dims& d) {
    return std::max(bwd_workspace_bytes_for(d, false, true, true, true), bwd_workspace_bytes_for(d, true, true, true, true));
}

// --------------------------------------------------------------- W and Y of one source point
// A zero row read in place of g blocks outside the energy grid, so the loads of
// a batch of frequencies can all be issued before their products (never written;
// not const, so it shares the global address space with g).
__device__ double bwd_zero_row[2] = {0.0, 0.0};

// Y_ij[x] for all nine (i,j), summed over every qz and the frequencies
// w in [w_lo, w_hi] of the 2*Nqz*Nw shifted g blocks (both energy branches);
// the loads of two qz and kBatch frequencies are in flight together.
// conj(alpha) is applied by the caller.  SIGNED: the g block at E'+w takes the
// table sDn (coefficients at +w), the one at E'-w the table sDm (at -w).
template <bool SIGNED>
__device__ __forceinline__ void compute_y(const Dims& d, const double* __restrict__ gS, int64_t a, int64_t kp,
                                          int64_t ep, const cd* sDn, const cd* sDm, int64_t w_lo, int64_t w_hi,
                                          int x, cd* y) {
    constexpr int kBatch = 5, kQ = 2;
#pragma unroll
    for (int ij = 0; ij < 9; ++ij) y[ij] = cd{0.0, 0.0};
    for (int64_t q0 = 0; q0 < d.nqz; q0 += kQ) {
        for (int64_t w0 = w_lo; w0 <= w_hi; w0 += kBatch) {
            cd hi[kQ][kBatch], lo[kQ][kBatch];
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                const bool q_in = q0 + u < d.nqz;
                const int64_t k = (kp + (q_in ? q0 + u : 0)) % d.nkz;
#pragma unroll
                for (int t = 0; t < kBatch; ++t) {
                    const int64_t w = w0 + t;
                    const bool in = q_in && w <= w_hi, h_ok = in && ep + w < d.ne, l_ok = in && ep - w >= 0;
                    // energies clamped to the source energy when out of the grid, so no pointer leaves g
                    const double* ph = h_ok ? gS + 2 * (off_S(d, k, h_ok ? ep + w : ep, a) + x) : bwd_zero_row;
                    const double* pl = l_ok ? gS + 2 * (off_S(d, k, l_ok ? ep - w : ep, a) + x) : bwd_zero_row;
                    hi[u][t] = cd{ph[0], ph[1]};
                    lo[u][t] = cd{pl[0], pl[1]};
                }
            }
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                if (q0 + u >= d.nqz) break;
#pragma unroll
                for (int t = 0; t < kBatch; ++t) {
                    const int64_t w = w0 + t;
                    if (w > w_hi) break;
                    const int64_t qw = ((q0 + u) * d.nw + (w - 1)) * 9;
                    if constexpr (SIGNED) {
#pragma unroll
                        for (int ij = 0; ij < 9; ++ij) {
                            cfma_conja(y[ij], sDn[qw + ij], hi[u][t]);
                            cfma_conja(y[ij], sDm[qw + ij], lo[u][t]);
                        }
                    } else {
                        const cd wv{hi[u][t].re + lo[u][t].re, hi[u][t].im + lo[u][t].im};
#pragma unroll
                        for (int ij = 0; ij < 9; ++ij) cfma_conja(y[ij], sDn[qw + ij], wv);
                    }
                }
            }
        }
    }
}

// --------------------------------------------------------------- dG and d gradH
template <bool SIGNED>
__global__ __launch_bounds__(kBwdThreads) void bwd_dg_dh_kernel(Dims d, const double* __restrict__ G,
                                                                const double* __restrict__ Dg,
                                                                const double* __restrict__ Dmg,
                                                                const double* __restrict__ Ag,
                                                                const double* __restrict__ gS, cd calpha,
                                                                const int32_t* __restrict__ offset,
                                                                const int32_t* __restrict__ edges,
                                                                const int32_t* __restrict__ order,
                                                                double* __restrict__ dG, double* __restrict__ dApart) {
    extern __shared__ double smem[];
    const int N = (int)d.norb, NN = N * N;
    const int nqw = (int)(d.nqz * d.nw);
    cd* sDn = reinterpret_cast<cd*>(smem);  // [q][w][ij]
    cd* sDm = sDn + nqw * 9;                // [q][w][ij]  (SIGNED: the coefficients at -w)
    cd* sA = sDm + (SIGNED ? nqw * 9 : 0);  // [3][N][N]   grad H of the edge
    cd* sY = sA + 3 * NN;                   // [9][N][N]
    cd* sB = sY + 9 * NN;                   // [N][N]
    cd* sT = sB + NN;                       // [3][N][N]   sum_i A_i^H Y_ij
    cd* sC = sT + 3 * NN;                   // [3][N][N]   A_j B^H
    cd* sE = sC + 3 * NN;                   // [3][N][N]   A_i B
    cd* sdA = sE + 3 * NN;                  // [3][N][N]   accumulated d gradH of the edge
    cd* sY1 = sT;                           // [9][N][N]   second half of the frequency sum of Y; shares
                                            // sT, sC, sE (9 N^2), which are written only after the merge
    const int tid = threadIdx.x;
    // One workgroup per (neighbour atom b, momentum k'): Nkz times as many
    // workgroups as atoms.  The Nkz workgroups of one atom get ids on the same
    // XCD (they read the same D, grad H and g blocks); the atoms come in
    // decreasing in-degree (a workgroup walks the edges into its atom), so the
    // longest workgroups start first.
    const int64_t bid = blockIdx.x, span = 8 * d.nkz;
    const int64_t pos = (bid / span) * 8 + bid % 8;
    const int64_t kp = (bid % span) / 8;
    if (pos >= d.na) return;  // uniform for the workgroup, before any barrier
    const int64_t b = order[pos];
    const int32_t e_lo = offset[b], e_hi = offset[b + 1];

    // slots >= 1 of dG are not read by the forward map: zero
    if (dG && (d.gs > 1 || e_lo == e_hi)) {
        for (int64_t ep = 0; ep < d.ne; ++ep) {
            const int64_t base = off_G(d, kp, ep, b);
            const int64_t from = (e_lo == e_hi) ? 0 : NN;
            for (int64_t x = from + tid; x < d.gs * NN; x += kBwdThreads) cstore(dG, base + x, cd{0.0, 0.0});
        }
    }
    for (int32_t ei = e_lo; ei < e_hi; ++ei) {
        const int32_t edge = edges[ei];
        const int64_t a = edge / d.nb, n = edge % d.nb;
        __syncthreads();
        for (int x = tid; x < nqw * 9; x += kBwdThreads) {
            const int ij = x % 9, qw = x / 9;
            sDn[x] = cload(Dg, off_D(d, qw / d.nw, qw % d.nw, a, n) + ij);
            if constexpr (SIGNED) sDm[x] = cload(Dmg, off_D(d, qw / d.nw, qw % d.nw, a, n) + ij);
        }
        for (int x = tid; x < 3 * NN; x += kBwdThreads) {
            sA[x] = cload(Ag, off_A(d, a, n, 0) + x);
            sdA[x] = cd{0.0, 0.0};
        }
        __syncthreads();
        for (int64_t ep = 0; ep < d.ne; ++ep) {
            // Y: threads [0, NN) sum the frequencies up to Nw/2, threads
            // [kYHalf, kYHalf + NN) the rest; the halves are then added
            const int yh = tid >= kYHalf ? 1 : 0;
            for (int yx = tid - yh * kYHalf; yx < NN; yx += kYHalf) {
                cd y[9];
                const int64_t w_mid = d.nw / 2;
                compute_y<SIGNED>(d, gS, a, kp, ep, sDn, sDm, yh ? w_mid + 1 : 1, yh ? d.nw : w_mid, yx, y);
                cd* dst = yh ? sY1 : sY;
#pragma unroll
                for (int ij = 0; ij < 9; ++ij) dst[ij * NN + yx] = y[ij];
                if (!yh) sB[yx] = cload(G, off_G(d, kp, ep, b) + yx);
            }
            __syncthreads();
            for (int x = tid; x < 9 * NN; x += kBwdThreads) {
                const cd u = sY[x], v = sY1[x];
                sY[x] = cmul(calpha, cd{u.re + v.re, u.im + v.im});
            }
            __syncthreads();
            // T_j = sum_i A_i^H Y_ij ; C_j = A_j B^H ; E_i = A_i B
            for (int x = tid; x < 9 * NN; x += kBwdThreads) {
                const int m = x / NN, rc = x % NN, r = rc / N, c = rc % N;
                cd s{0.0, 0.0};
                if (m < 3) {
                    const int j = m;
                    for (int i = 0; i < 3; ++i)
                        for (int t = 0; t < N; ++t) cfma_conja(s, sA[i * NN + t * N + r], sY[(i * 3 + j) * NN + t * N + c]);
                    sT[j * NN + rc] = s;
                } else if (m < 6) {
                    const int j = m - 3;
                    for (int t = 0; t < N; ++t) cfma_conj(s, sA[j * NN + r * N + t], sB[c * N + t]);
                    sC[j * NN + rc] = s;
                } else {
                    const int i = m - 6;
                    for (int t = 0; t < N; ++t) cfma(s, sA[i * NN + r * N + t], sB[t * N + c]);
                    sE[i * NN + rc] = s;
                }
            }
            __syncthreads();
            // dG[k',E',b] (+)= sum_j T_j A_j
            for (int x = tid; dG && x < NN; x += kBwdThreads) {
                const int t = x / N, u = x % N;
                cd s{0.0, 0.0};
                for (int j = 0; j < 3; ++j)
                    for (int c = 0; c < N; ++c) cfma(s, sT[j * NN + t * N + c], sA[j * NN + c * N + u]);
                const int64_t o = off_G(d, kp, ep, b) + x;
                if (ei != e_lo) {
                    const cd prev = cload(dG, o);
                    s.re += prev.re;
                    s.im += prev.im;
                }
                cstore(dG, o, s);
            }
            // d gradH_m += sum_j Y_mj C_j + sum_i Y_im^H E_i
            for (int x = tid; dApart && x < 3 * NN; x += kBwdThreads) {
                const int m = x / NN, rc = x % NN, r = rc / N, c = rc % N;
                cd s = sdA[x];
                for (int j = 0; j < 3; ++j)
                    for (int t = 0; t < N; ++t) cfma(s, sY[(m * 3 + j) * NN + r * N + t], sC[j * NN + t * N + c]);
                for (int i = 0; i < 3; ++i)
                    for (int t = 0; t < N; ++t) cfma_conja(s, sY[(i * 3 + m) * NN + t * N + r], sE[i * NN + t * N + c]);
                sdA[x] = s;
            }
            __syncthreads();
        }
        // this momentum's share of the edge's d gradH (edge index a * nb + n)
        for (int x = tid; dApart && x < 3 * NN; x += kBwdThreads)
            cstore(dApart, (kp * d.na * d.nb + edge) * 3 * NN + x, sdA[x]);
    }
}

// d gradH of every edge (a, n): its partial sums (one per momentum k', or per
// energy range on the matrix-core path) added in share order; an edge whose
// neighbour entry lies outside [0, na) has no terms and gets zero
__global__ void bwd_dh_reduce_kernel(Dims d, const int32_t* __restrict__ nbr, const double* __restrict__ dApart,
                                     int64_t shares, double* __restrict__ dA) {
    const int64_t NN3 = 3 * d.norb * d.norb, per_k = d.na * d.nb * NN3;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < per_k; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = nbr[x / NN3];
        cd s{0.0, 0.0};
        if (b >= 0 && b < d.na)
            for (int64_t kp = 0; kp < shares; ++kp) {
                const cd v = cload(dApart, kp * per_k + x);
                s.re += v.re;
                s.im += v.im;
            }
        cstore(dA, x, s);
    }
}

// --------------------------------------------------------------- dD
// branches: bit 0 the g blocks at E'+w (the terms with G at E - w), bit 1 those at E'-w
__global__ __launch_bounds__(kBwdThreads) void bwd_dd_kernel(Dims d, const double* __restrict__ G,
                                                             const double* __restrict__ Ag,
                                                             const int32_t* __restrict__ nbr,
                                                             const double* __restrict__ gS, cd calpha, int branches,
                                                             double* __restrict__ dD) {
    extern __shared__ double smem[];
    const int N = (int)d.norb, NN = N * N;
    const int nqw = (int)(d.nqz * d.nw);
    cd* sA = reinterpret_cast<cd*>(smem);  // [3][N][N]
    cd* sB = sA + 3 * NN;                  // [N][N]
    cd* sE = sB + NN;                      // [3][N][N]  A_i B
    cd* sP = sE + 3 * NN;                  // [9][N][N]  A_i B A_j^H
    const int tid = threadIdx.x;
    const int64_t edge = blockIdx.x;
    if (edge >= d.na * d.nb) return;
    const int64_t a = edge / d.nb, n = edge % d.nb;
    const int32_t b = nbr[edge];
    for (int x = tid; x < 3 * NN; x += kBwdThreads) sA[x] = cload(Ag, off_A(d, a, n, 0) + x);
    // each thread owns up to two (q, w) pairs and accumulates all nine (i,j)
    constexpr int kPer = 2;
    cd acc[kPer][9];
#pragma unroll
    for (int s = 0; s < kPer; ++s)
#pragma unroll
        for (int ij = 0; ij < 9; ++ij) acc[s][ij] = cd{0.0, 0.0};
    const bool valid_b = b >= 0 && b < d.na;
    for (int64_t kp = 0; kp < d.nkz; ++kp)
        for (int64_t ep = 0; ep < d.ne; ++ep) {
            __syncthreads();
            for (int x = tid; x < NN; x += kBwdThreads) sB[x] = valid_b ? cload(G, off_G(d, kp, ep, b) + x) : cd{0.0, 0.0};
            __syncthreads();
            for (int x = tid; x < 3 * NN; x += kBwdThreads) {
                const int i = x / NN, r = (x % NN) / N, c = x % N;
                cd s{0.0, 0.0};
                for (int t = 0; t < N; ++t) cfma(s, sA[i * NN + r * N + t], sB[t * N + c]);
                sE[x] = s;
            }
            __syncthreads();
            for (int x = tid; x < 9 * NN; x += kBwdThreads) {
                const int ij = x / NN, i = ij / 3, j = ij % 3, r = (x % NN) / N, c = x % N;
                cd s{0.0, 0.0};
                for (int u = 0; u < N; ++u) cfma_conj(s, sE[i * NN + r * N + u], sA[j * NN + c * N + u]);
                sP[x] = s;
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                const int qw = tid + s * kBwdThreads;
                if (qw < nqw) {
                    const int64_t q = qw / d.nw, w = qw % d.nw + 1;
                    const int64_t k = (kp + q) % d.nkz;
                    const bool hi = (branches & 1) && ep + w < d.ne, lo = (branches & 2) && ep - w >= 0;
                    const double* g1 = gS + 2 * off_S(d, k, hi ? ep + w : ep, a);
                    const double* g2 = gS + 2 * off_S(d, k, lo ? ep - w : ep, a);
                    for (int rc = 0; rc < NN; ++rc) {
                        cd wv{0.0, 0.0};
                        if (hi) {
                            const cd v = cload(g1, rc);
                            wv.re += v.re;
                            wv.im += v.im;
                        }
                        if (lo) {
                            const cd v = cload(g2, rc);
                            wv.re += v.re;
                            wv.im += v.im;
                        }
#pragma unroll
                        for (int ij = 0; ij < 9; ++ij) cfma_conja(acc[s][ij], sP[ij * NN + rc], wv);
                    }
                }
            }
        }
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
        const int qw = tid + s * kBwdThreads;
        if (qw < nqw) {
            const int64_t q = qw / d.nw, w = qw % d.nw;
#pragma unroll
            for (int ij = 0; ij < 9; ++ij) cstore(dD, off_D(d, q, w, a, n) + ij, cmul(calpha, acc[s][ij]));
        }
    }
}

static size_t bwd_lds_dg(const Dims& d, bool signed_form = false) {
    const size_t NN = (size_t)(d.norb * d.norb);
    return sizeof(cd) * ((size_t)d.nqz * d.nw * 9 * (signed_form ? 2 : 1) + 3 * NN + 9 * NN + NN + 4 * 3 * NN);
}
static size_t bwd_lds_dd(const Dims& d) {
    const size_t NN = (size_t)(d.norb * d.norb);
    return sizeof(cd) * (3 * NN + NN + 3 * NN + 9 * NN);
}

bool bwd_supported(const Dims& d) {
    return d.nqz * d.nw <= 2 * kBwdThreads && d.norb * d.norb <= kBwdThreads && bwd_lds_dg(d, true) <= 160 * 1024 &&
           bwd_lds_dd(d) <= 160 * 1024 && d.na * d.nb <= INT32_MAX && (d.na + 7) / 8 * 8 * d.nkz <= INT32_MAX;
}

// dD (or dDp / dDm) for the given energy branches (gT: the atom-major copy of gS, or NULL)
static hipError_t launch_dd(const Dims& d, const double* G, const double* A, const int32_t* nbr, const double* gS,
                            const double* gT, cd calpha, double* dD, int branches, hipStream_t stream) {
    if (pse_mfma_specialised(d)) return launch_dd_mfma(d, G, A, nbr, gS, gT, calpha, dD, stream, branches);
    const size_t lds = bwd_lds_dd(d);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(bwd_dd_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bwd_dd_kernel, dim3((unsigned)(d.na * d.nb)), dim3(kBwdThreads), lds, stream, d, G, A, nbr, gS,
                       calpha, branches, dD);
    return hipGetLastError();
}

hipError_t launch_bwd(const Dims& d, const double* G, const double* Dp, const double* Dm, const double* A,
                      const int32_t* nbr, cd alpha, const double* gS, double* dG, double* dDp, double* dDm, double* dA,
                      void* ws, hipStream_t stream, bool signed_form, bool copy_g) {
    const cd calpha{alpha.re, -alpha.im};
    const bool mfma = bwd_use_mfma(d, signed_form);
    // every attribute is set before the first launch, so a failure leaves all outputs untouched
    const size_t lds = bwd_lds_dg(d, signed_form);
    auto kern = signed_form ? bwd_dg_dh_kernel<true> : bwd_dg_dh_kernel<false>;
    if (dG || dA) {
        hipError_t e = mfma ? bwd_mfma_prepare()
                            : hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if ((dDp || dDm) && !pse_mfma_specialised(d)) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(bwd_dd_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwd_lds_dd(d));
        if (e != hipSuccess) return e;
    }
    if (dG || dA) {
        int32_t* count = reinterpret_cast<int32_t*>(ws);
        int32_t* offset = count + d.na;
        int32_t* cursor = offset + d.na + 1;
        int32_t* edges = cursor + d.na;
        const unsigned g1 = (unsigned)((d.na * d.nb + 255) / 256 < 4096 ? (d.na * d.nb + 255) / 256 : 4096);
        hipLaunchKernelGGL(zero_i32_kernel, dim3(g1), dim3(256), 0, stream, d.na, count);
        hipLaunchKernelGGL(rcsr_count_kernel, dim3(g1), dim3(256), 0, stream, d.na, d.nb, nbr, count);
        hipLaunchKernelGGL(rcsr_scan_kernel, dim3(1), dim3(1024), 0, stream, d.na, count, offset, cursor);
        hipLaunchKernelGGL(rcsr_fill_kernel, dim3(g1), dim3(256), 0, stream, d.na, d.nb, nbr, cursor, edges);
        const unsigned g2 = (unsigned)((d.na + 255) / 256 < 4096 ? (d.na + 255) / 256 : 4096);
        hipLaunchKernelGGL(rcsr_sort_kernel, dim3(g2), dim3(256), 0, stream, d.na, offset, edges);
        int32_t* order = edges + d.na * d.nb;
        hipLaunchKernelGGL(rcsr_order_kernel, dim3(1), dim3(1024), 0, stream, d.na, count, order);
        double* dApart = dA ? reinterpret_cast<double*>(reinterpret_cast<char*>(ws) + bwd_csr_bytes(d)) : nullptr;
        hipError_t e;
        if (mfma) {
            e = launch_bwd_mfma(d, G, Dp, A, gS, calpha, offset, edges, order, dG, dApart, stream);
        } else {
            const int64_t groups = (d.na + 7) / 8 * 8 * d.nkz;
            hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(kBwdThreads), lds, stream, d, G, Dp, Dm, A, gS,
                               calpha, offset, edges, order, dG, dApart);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
        if (dA) {
            const int64_t n = d.na * d.nb * 3 * d.norb * d.norb;
            const unsigned g3 = (unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
            hipLaunchKernelGGL(bwd_dh_reduce_kernel, dim3(g3), dim3(256), 0, stream, d, nbr, dApart,
                               bwd_shares(d, signed_form), dA);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    if (signed_form ? !dDp && !dDm : !dDp) return hipGetLastError();
    // the matrix-core D gradient reads g from its atom-major copy when the workspace holds one
    double* gT = nullptr;
    if (copy_g && !signed_form && pse_atom_major_bytes(d) > 0) {
        gT = reinterpret_cast<double*>(reinterpret_cast<char*>(ws) + bwd_csr_bytes(d) +
                                       (dA ? bwd_dh_bytes(d, signed_form) : 0));
        hipError_t e = pse_atom_major_g(d, gS, gT, stream);
        if (e != hipSuccess) return e;
    }
    if (!signed_form) return launch_dd(d, G, A, nbr, gS, gT, calpha, dDp, 3, stream);
    if (dDp) {
        hipError_t e = launch_dd(d, G, A, nbr, gS, gT, calpha, dDp, 1, stream);
        if (e != hipSuccess) return e;
    }
    if (dDm) return launch_dd(d, G, A, nbr, gS, gT, calpha, dDm, 2, stream);
    return hipGetLastError();
}

}  // namespace sse
