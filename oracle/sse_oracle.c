/*
 * CPU oracle for the electron-phonon scattering self-energy (SSE).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header or table with the HIP implementation.
 *
 * What it computes (Eq. 3 of Ziogas et al., SC'19, "Current State of the Art",
 * with the readings listed in the design notes):
 *
 *   Sigma[k,e,a] = alpha * sum_{q=0}^{Nqz-1} sum_{m=1}^{Nw} sum_{s=+1,-1}
 *                  [0 <= e - s*m < NE] * sum_{n=0}^{NB-1} sum_{i,j=0}^{2}
 *                  D[q, m-1, a, n, i, j] * A[a,n,i] . G[(k-q) mod Nkz, e-s*m, nbr[a,n], 0]
 *                                        . A[a,n,j]^H
 *
 * The *_signed functions take one table per sign of the frequency: the s = +1
 * terms (G at e - m) read Dp[q, m-1, ...] (coefficient at +w_m), the s = -1
 * terms (G at e + m) read Dm[q, m-1, ...] (coefficient at -w_m), which is the
 * integral of Eq. 3 over signed frequencies on a grid of Nw positive ones.
 *
 * A[a,n,i] is grad_i H for the pair (a, b = nbr[a,n]); grad_j H_ba = A[a,n,j]^H
 * because H is Hermitian.  The *_ex functions also take the stored blocks
 * Aba[a,n,j] = grad_j H_ba (layout of A) as the right factor of Eq. 3 in place
 * of A[a,n,j]^H; a NULL Aba means the Hermitian reading.  Every product is an Norb x Norb complex matrix
 * product; D[...,i,j] is a complex scalar; only the diagonal block of Sigma is
 * formed (the paper keeps only the diagonal blocks of the electron SSE).
 *
 * The loop nest below follows that sum term by term, in fp64, with no
 * blocking or reordering.  The only liberty taken is that T = A_i . G_b is
 * formed once per (term, i) and used for the three j's; this changes no
 * arithmetic result.
 *
 * Layouts (row-major, complex = interleaved (re, im) doubles):
 *   G   [nkz][ne][na][g_slots][norb][norb]
 *   D   [nqz][nw][na][nb][3][3]
 *   A   [na][nb][3][norb][norb]      (grad H)
 *   nbr [na][nb]                    int32
 *   Sigma, dSigma [nkz][ne][na][norb][norb]
 *
 * dims[] = {nkz, ne, nqz, nw, na, nb, norb, g_slots}.  The oracle requires
 * nqz == nkz (the two momentum grids coincide, Sec. "Scalability").
 *
 * Return codes: 0 ok, 1 null pointer, 2 bad dims, 6 neighbour out of range.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;

static inline cplx c_mul(cplx x, cplx y) {
    cplx r = { x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re };
    return r;
}
static inline cplx c_conj(cplx x) { cplx r = { x.re, -x.im }; return r; }
static inline cplx c_add(cplx x, cplx y) { cplx r = { x.re + y.re, x.im + y.im }; return r; }
static inline cplx c_at(const double* p, int64_t idx) { cplx r = { p[2 * idx], p[2 * idx + 1] }; return r; }

typedef struct {
    int64_t nkz, ne, nqz, nw, na, nb, norb, gs;
} odims;

static int read_dims(const int64_t* d, odims* o) {
    if (!d) return 1;
    o->nkz = d[0]; o->ne = d[1]; o->nqz = d[2]; o->nw = d[3];
    o->na = d[4]; o->nb = d[5]; o->norb = d[6]; o->gs = d[7];
    if (o->nkz <= 0 || o->ne <= 0 || o->nqz <= 0 || o->nw <= 0 || o->na <= 0 ||
        o->nb <= 0 || o->norb <= 0 || o->gs <= 0)
        return 2;
    if (o->nqz != o->nkz) return 2;
    return 0;
}

static int check_nbr(const odims* d, const int32_t* nbr) {
    for (int64_t x = 0; x < d->na * d->nb; ++x)
        if (nbr[x] < 0 || nbr[x] >= d->na) return 6;
    return 0;
}

/* flat offsets (in complex elements) */
static inline int64_t off_G(const odims* d, int64_t k, int64_t e, int64_t b) {
    return (((k * d->ne + e) * d->na + b) * d->gs + 0) * d->norb * d->norb;
}
static inline int64_t off_D(const odims* d, int64_t q, int64_t w, int64_t a, int64_t n, int i, int j) {
    return ((((q * d->nw + w) * d->na + a) * d->nb + n) * 3 + i) * 3 + j;
}
static inline int64_t off_A(const odims* d, int64_t a, int64_t n, int i) {
    return ((a * d->nb + n) * 3 + i) * d->norb * d->norb;
}
static inline int64_t off_S(const odims* d, int64_t k, int64_t e, int64_t a) {
    return ((k * d->ne + e) * d->na + a) * d->norb * d->norb;
}

/* out = X . Y   (N x N complex) */
static void mat_mul(int64_t N, const double* X, const double* Y, cplx* out) {
    for (int64_t r = 0; r < N; ++r)
        for (int64_t c = 0; c < N; ++c) {
            cplx s = { 0.0, 0.0 };
            for (int64_t t = 0; t < N; ++t) s = c_add(s, c_mul(c_at(X, r * N + t), c_at(Y, t * N + c)));
            out[r * N + c] = s;
        }
}

/* acc[r][c] += d * (T . Y^H)[r][c] */
static void acc_mul_adj(int64_t N, cplx d, const cplx* T, const double* Y, cplx* acc) {
    for (int64_t r = 0; r < N; ++r)
        for (int64_t c = 0; c < N; ++c) {
            cplx s = { 0.0, 0.0 };
            for (int64_t u = 0; u < N; ++u) s = c_add(s, c_mul(T[r * N + u], c_conj(c_at(Y, c * N + u))));
            acc[r * N + c] = c_add(acc[r * N + c], c_mul(d, s));
        }
}

/* acc[r][c] += d * (T . Y)[r][c] */
static void acc_mul(int64_t N, cplx d, const cplx* T, const double* Y, cplx* acc) {
    for (int64_t r = 0; r < N; ++r)
        for (int64_t c = 0; c < N; ++c) {
            cplx s = { 0.0, 0.0 };
            for (int64_t u = 0; u < N; ++u) s = c_add(s, c_mul(T[r * N + u], c_at(Y, u * N + c)));
            acc[r * N + c] = c_add(acc[r * N + c], c_mul(d, s));
        }
}

/* One output block Sigma[k,e,a] (Eq. 3), written to out as N*N complex.
 * Eq. 3 integrates over signed frequencies; with the Nw stored frequencies
 * w_m > 0 the s = +1 terms (G at e - m) carry the coefficient at +w_m (Dp) and
 * the s = -1 terms (G at e + m) the coefficient at -w_m (Dm).  The one-table
 * form reads the same table for both (Dm == Dp).  The right factor is
 * grad_j H_ba: Aba[a,n,j] when given, else A[a,n,j]^H. */
static void sigma_block(const odims* d, const double* G, const double* Dp, const double* Dm, const double* A,
                        const double* Aba, const int32_t* nbr, cplx alpha, int64_t k, int64_t e, int64_t a,
                        cplx* acc, cplx* T, double* out) {
    const int64_t N = d->norb;
    for (int64_t x = 0; x < N * N; ++x) { acc[x].re = 0.0; acc[x].im = 0.0; }
    for (int64_t q = 0; q < d->nqz; ++q) {
        const int64_t kp = ((k - q) % d->nkz + d->nkz) % d->nkz;
        for (int64_t m = 1; m <= d->nw; ++m) {
            for (int s = +1; s >= -1; s -= 2) {
                const int64_t ep = e - s * m;
                if (ep < 0 || ep >= d->ne) continue;
                const double* D = s > 0 ? Dp : Dm;
                for (int64_t n = 0; n < d->nb; ++n) {
                    const int64_t b = nbr[a * d->nb + n];
                    const double* Gb = G + 2 * off_G(d, kp, ep, b);
                    for (int i = 0; i < 3; ++i) {
                        mat_mul(N, A + 2 * off_A(d, a, n, i), Gb, T);
                        for (int j = 0; j < 3; ++j) {
                            const cplx dij = c_at(D, off_D(d, q, m - 1, a, n, i, j));
                            if (Aba)
                                acc_mul(N, dij, T, Aba + 2 * off_A(d, a, n, j), acc);
                            else
                                acc_mul_adj(N, dij, T, A + 2 * off_A(d, a, n, j), acc);
                        }
                    }
                }
            }
        }
    }
    for (int64_t x = 0; x < N * N; ++x) {
        cplx v = c_mul(alpha, acc[x]);
        out[2 * x] = v.re;
        out[2 * x + 1] = v.im;
    }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sigma at a list of output points pts[p] = (k, e, a); out is [npts][norb][norb].
 * Dp: coefficients at +w (terms with G at e - m), Dm: at -w (G at e + m);
 * Aba: stored grad_j H_ba blocks, or NULL for A^H. */
int oracle_sse_points_ex(const int64_t* dims, const double* G, const double* Dp, const double* Dm,
                         const double* A, const double* Aba, const int32_t* nbr, double alpha_re, double alpha_im,
                         int64_t npts, const int64_t* pts, double* out) {
    odims d;
    int rc = read_dims(dims, &d);
    if (rc) return rc;
    if (!G || !Dp || !Dm || !A || !nbr || (npts > 0 && (!pts || !out))) return 1;
    if ((rc = check_nbr(&d, nbr))) return rc;
    for (int64_t p = 0; p < npts; ++p)
        if (pts[3 * p] < 0 || pts[3 * p] >= d.nkz || pts[3 * p + 1] < 0 || pts[3 * p + 1] >= d.ne ||
            pts[3 * p + 2] < 0 || pts[3 * p + 2] >= d.na)
            return 2;
    const cplx alpha = { alpha_re, alpha_im };
    const int64_t NN = d.norb * d.norb;
    int fail = 0;
#pragma omp parallel
    {
        cplx* acc = (cplx*)malloc(sizeof(cplx) * NN);
        cplx* T = (cplx*)malloc(sizeof(cplx) * NN);
        if (!acc || !T) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t p = 0; p < npts; ++p)
                sigma_block(&d, G, Dp, Dm, A, Aba, nbr, alpha, pts[3 * p], pts[3 * p + 1], pts[3 * p + 2], acc, T,
                            out + 2 * NN * p);
        }
        free(acc);
        free(T);
    }
    return fail ? 7 : 0;
}

/* One table per sign of the frequency, Hermitian reading of grad_j H_ba. */
int oracle_sse_points_signed(const int64_t* dims, const double* G, const double* Dp, const double* Dm,
                             const double* A, const int32_t* nbr, double alpha_re, double alpha_im,
                             int64_t npts, const int64_t* pts, double* out) {
    return oracle_sse_points_ex(dims, G, Dp, Dm, A, NULL, nbr, alpha_re, alpha_im, npts, pts, out);
}

/* The one-table form: the same coefficient table for both signs of the frequency. */
int oracle_sse_points(const int64_t* dims, const double* G, const double* D, const double* A,
                      const int32_t* nbr, double alpha_re, double alpha_im, int64_t npts,
                      const int64_t* pts, double* out) {
    return oracle_sse_points_ex(dims, G, D, D, A, NULL, nbr, alpha_re, alpha_im, npts, pts, out);
}

/* Full Sigma [nkz][ne][na][norb][norb]; Dp, Dm and Aba as for oracle_sse_points_ex. */
int oracle_sse_forward_ex(const int64_t* dims, const double* G, const double* Dp, const double* Dm,
                          const double* A, const double* Aba, const int32_t* nbr, double alpha_re,
                          double alpha_im, double* Sigma) {
    odims d;
    int rc = read_dims(dims, &d);
    if (rc) return rc;
    if (!G || !Dp || !Dm || !A || !nbr || !Sigma) return 1;
    if ((rc = check_nbr(&d, nbr))) return rc;
    const cplx alpha = { alpha_re, alpha_im };
    const int64_t NN = d.norb * d.norb;
    const int64_t nblk = d.nkz * d.ne * d.na;
    int fail = 0;
#pragma omp parallel
    {
        cplx* acc = (cplx*)malloc(sizeof(cplx) * NN);
        cplx* T = (cplx*)malloc(sizeof(cplx) * NN);
        if (!acc || !T) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int64_t x = 0; x < nblk; ++x) {
                const int64_t a = x % d.na, e = (x / d.na) % d.ne, k = x / (d.na * d.ne);
                sigma_block(&d, G, Dp, Dm, A, Aba, nbr, alpha, k, e, a, acc, T, Sigma + 2 * off_S(&d, k, e, a));
            }
        }
        free(acc);
        free(T);
    }
    return fail ? 7 : 0;
}

/* Full Sigma over signed frequencies, Hermitian reading of grad_j H_ba. */
int oracle_sse_forward_signed(const int64_t* dims, const double* G, const double* Dp, const double* Dm,
                              const double* A, const int32_t* nbr, double alpha_re, double alpha_im,
                              double* Sigma) {
    return oracle_sse_forward_ex(dims, G, Dp, Dm, A, NULL, nbr, alpha_re, alpha_im, Sigma);
}

/* Full Sigma, one-table form (the same table for both signs of the frequency). */
int oracle_sse_forward(const int64_t* dims, const double* G, const double* D, const double* A,
                       const int32_t* nbr, double alpha_re, double alpha_im, double* Sigma) {
    return oracle_sse_forward_ex(dims, G, D, D, A, NULL, nbr, alpha_re, alpha_im, Sigma);
}

/*
 * Adjoint of the map above for a real scalar L, with PyTorch's convention for
 * complex gradients (grad = dL/dRe z + i dL/dIm z).  Given gS = dL/dSigma,
 * each valid term t = (k,e,a,q,m,s,n,i,j) with d = D[q,m-1,a,n,i,j],
 * A_i = A[a,n,i], B = G[k',e',b,0] and g = gS[k,e,a] contributes
 *   dG[k',e',b,0]        += conj(alpha d) A_i^H g A_j
 *   dD[q,m-1,a,n,i,j]    += conj(alpha) sum_{rc} conj((A_i B A_j^H)[r,c]) g[r,c]
 *   dA[a,n,i]            += conj(alpha d) g A_j B^H
 *   dA[a,n,j]            += alpha d g^H A_i B
 * (derived from dL = Re <g, dSigma>).  dG slots >= 1 are not read by the
 * forward map and are set to zero.  Any of dG, dD, dA may be NULL.
 * Over signed frequencies the s = +1 terms read Dp and feed dDp, the s = -1
 * terms read Dm and feed dDm (the one-table form passes the same table and the
 * same gradient array for both).
 */
static void adjoint_terms_for_atom(const odims* d, const double* G, const double* Dp, const double* Dm,
                                   const double* A, const int32_t* nbr, cplx alpha, const double* gS, int64_t a,
                                   double* dDp, double* dDm, double* dA, cplx* work) {
    const int64_t N = d->norb, NN = N * N;
    cplx* P = work;          /* A_i B A_j^H */
    cplx* X = work + NN;     /* A_i B       */
    cplx* Y = work + 2 * NN; /* g A_j       */
    cplx* Z = work + 3 * NN; /* g^H A_i     */
    const cplx calpha = c_conj(alpha);
    for (int64_t k = 0; k < d->nkz; ++k)
        for (int64_t e = 0; e < d->ne; ++e) {
            const double* g = gS + 2 * off_S(d, k, e, a);
            for (int64_t q = 0; q < d->nqz; ++q) {
                const int64_t kp = ((k - q) % d->nkz + d->nkz) % d->nkz;
                for (int64_t m = 1; m <= d->nw; ++m)
                    for (int s = +1; s >= -1; s -= 2) {
                        const int64_t ep = e - s * m;
                        if (ep < 0 || ep >= d->ne) continue;
                        const double* D = s > 0 ? Dp : Dm;
                        double* dD = s > 0 ? dDp : dDm;
                        for (int64_t n = 0; n < d->nb; ++n) {
                            const int64_t b = nbr[a * d->nb + n];
                            const double* B = G + 2 * off_G(d, kp, ep, b);
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j) {
                                    const double* Ai = A + 2 * off_A(d, a, n, i);
                                    const double* Aj = A + 2 * off_A(d, a, n, j);
                                    const cplx dij = c_at(D, off_D(d, q, m - 1, a, n, i, j));
                                    const cplx ad = c_mul(alpha, dij);
                                    const cplx cad = c_conj(ad);
                                    mat_mul(N, Ai, B, X);
                                    if (dD) {
                                        /* P = X . A_j^H ; dD += conj(alpha) sum conj(P) g */
                                        cplx sacc = { 0.0, 0.0 };
                                        for (int64_t r = 0; r < N; ++r)
                                            for (int64_t c = 0; c < N; ++c) {
                                                cplx p = { 0.0, 0.0 };
                                                for (int64_t u = 0; u < N; ++u)
                                                    p = c_add(p, c_mul(X[r * N + u], c_conj(c_at(Aj, c * N + u))));
                                                P[r * N + c] = p;
                                                sacc = c_add(sacc, c_mul(c_conj(p), c_at(g, r * N + c)));
                                            }
                                        cplx v = c_mul(calpha, sacc);
                                        const int64_t o = off_D(d, q, m - 1, a, n, i, j);
                                        dD[2 * o] += v.re;
                                        dD[2 * o + 1] += v.im;
                                    }
                                    if (dA) {
                                        /* dA_i += conj(alpha d) g A_j B^H */
                                        for (int64_t r = 0; r < N; ++r)
                                            for (int64_t u = 0; u < N; ++u) {
                                                cplx y = { 0.0, 0.0 };
                                                for (int64_t t = 0; t < N; ++t)
                                                    y = c_add(y, c_mul(c_at(g, r * N + t), c_at(Aj, t * N + u)));
                                                Y[r * N + u] = y;
                                            }
                                        double* dAi = dA + 2 * off_A(d, a, n, i);
                                        for (int64_t r = 0; r < N; ++r)
                                            for (int64_t c = 0; c < N; ++c) {
                                                cplx v = { 0.0, 0.0 };
                                                for (int64_t u = 0; u < N; ++u)
                                                    v = c_add(v, c_mul(Y[r * N + u], c_conj(c_at(B, c * N + u))));
                                                v = c_mul(cad, v);
                                                dAi[2 * (r * N + c)] += v.re;
                                                dAi[2 * (r * N + c) + 1] += v.im;
                                            }
                                        /* dA_j += alpha d g^H A_i B  (= alpha d g^H X) */
                                        for (int64_t r = 0; r < N; ++r)
                                            for (int64_t u = 0; u < N; ++u) {
                                                cplx z = { 0.0, 0.0 };
                                                for (int64_t t = 0; t < N; ++t)
                                                    z = c_add(z, c_mul(c_conj(c_at(g, t * N + r)), X[t * N + u]));
                                                Z[r * N + u] = z;
                                            }
                                        double* dAj = dA + 2 * off_A(d, a, n, j);
                                        for (int64_t x = 0; x < NN; ++x) {
                                            cplx v = c_mul(ad, Z[x]);
                                            dAj[2 * x] += v.re;
                                            dAj[2 * x + 1] += v.im;
                                        }
                                    }
                                }
                        }
                    }
            }
        }
}

/* dG contributions landing on source atom b (terms whose neighbour is b). */
static void adjoint_dG_for_atom(const odims* d, const double* Dp, const double* Dm, const double* A,
                                const int32_t* nbr, cplx alpha, const double* gS, int64_t b, double* dG,
                                cplx* work) {
    const int64_t N = d->norb, NN = N * N;
    cplx* Y = work; /* A_i^H g */
    for (int64_t a = 0; a < d->na; ++a)
        for (int64_t n = 0; n < d->nb; ++n) {
            if (nbr[a * d->nb + n] != b) continue;
            for (int64_t k = 0; k < d->nkz; ++k)
                for (int64_t e = 0; e < d->ne; ++e) {
                    const double* g = gS + 2 * off_S(d, k, e, a);
                    for (int64_t q = 0; q < d->nqz; ++q) {
                        const int64_t kp = ((k - q) % d->nkz + d->nkz) % d->nkz;
                        for (int64_t m = 1; m <= d->nw; ++m)
                            for (int s = +1; s >= -1; s -= 2) {
                                const int64_t ep = e - s * m;
                                if (ep < 0 || ep >= d->ne) continue;
                                const double* D = s > 0 ? Dp : Dm;
                                double* dB = dG + 2 * off_G(d, kp, ep, b);
                                for (int i = 0; i < 3; ++i) {
                                    const double* Ai = A + 2 * off_A(d, a, n, i);
                                    for (int64_t t = 0; t < N; ++t)
                                        for (int64_t c = 0; c < N; ++c) {
                                            cplx y = { 0.0, 0.0 };
                                            for (int64_t r = 0; r < N; ++r)
                                                y = c_add(y, c_mul(c_conj(c_at(Ai, r * N + t)), c_at(g, r * N + c)));
                                            Y[t * N + c] = y;
                                        }
                                    for (int j = 0; j < 3; ++j) {
                                        const double* Aj = A + 2 * off_A(d, a, n, j);
                                        const cplx cad = c_conj(c_mul(alpha, c_at(D, off_D(d, q, m - 1, a, n, i, j))));
                                        for (int64_t t = 0; t < N; ++t)
                                            for (int64_t u = 0; u < N; ++u) {
                                                cplx v = { 0.0, 0.0 };
                                                for (int64_t c = 0; c < N; ++c)
                                                    v = c_add(v, c_mul(Y[t * N + c], c_at(Aj, c * N + u)));
                                                v = c_mul(cad, v);
                                                dB[2 * (t * N + u)] += v.re;
                                                dB[2 * (t * N + u) + 1] += v.im;
                                            }
                                    }
                                }
                            }
                    }
                }
        }
    (void)NN;
}

/* Adjoint over signed frequencies: gradients with respect to G, Dp, Dm and A.
 * dDp and dDm may be the same array (then it receives both); any output may be
 * NULL. */
int oracle_sse_backward_signed(const int64_t* dims, const double* G, const double* Dp, const double* Dm,
                               const double* A, const int32_t* nbr, double alpha_re, double alpha_im,
                               const double* dSigma, double* dG, double* dDp, double* dDm, double* dA) {
    odims d;
    int rc = read_dims(dims, &d);
    if (rc) return rc;
    if (!G || !Dp || !Dm || !A || !nbr || !dSigma || (!dDp) != (!dDm)) return 1;
    if ((rc = check_nbr(&d, nbr))) return rc;
    const cplx alpha = { alpha_re, alpha_im };
    const int64_t NN = d.norb * d.norb;
    if (dG) memset(dG, 0, sizeof(double) * 2 * d.nkz * d.ne * d.na * d.gs * NN);
    if (dDp) memset(dDp, 0, sizeof(double) * 2 * d.nqz * d.nw * d.na * d.nb * 9);
    if (dDm) memset(dDm, 0, sizeof(double) * 2 * d.nqz * d.nw * d.na * d.nb * 9);
    if (dA) memset(dA, 0, sizeof(double) * 2 * d.na * d.nb * 3 * NN);
    int fail = 0;
#pragma omp parallel
    {
        cplx* work = (cplx*)malloc(sizeof(cplx) * 4 * NN);
        if (!work) {
#pragma omp atomic write
            fail = 1;
        } else {
            if (dDp || dA) {
#pragma omp for schedule(dynamic, 1)
                for (int64_t a = 0; a < d.na; ++a)
                    adjoint_terms_for_atom(&d, G, Dp, Dm, A, nbr, alpha, dSigma, a, dDp, dDm, dA, work);
            }
            if (dG) {
#pragma omp for schedule(dynamic, 1)
                for (int64_t b = 0; b < d.na; ++b) adjoint_dG_for_atom(&d, Dp, Dm, A, nbr, alpha, dSigma, b, dG, work);
            }
        }
        free(work);
    }
    return fail ? 7 : 0;
}

/* The one-table form: both branches read D and feed dD. */
int oracle_sse_backward(const int64_t* dims, const double* G, const double* D, const double* A,
                        const int32_t* nbr, double alpha_re, double alpha_im, const double* dSigma,
                        double* dG, double* dD, double* dA) {
    return oracle_sse_backward_signed(dims, G, D, D, A, nbr, alpha_re, alpha_im, dSigma, dG, dD, dD, dA);
}

/*
 * The bracket of Eq. 3, D_ba - D_bb - D_aa + D_ab, for every pair (a, b = nbr[a,n]),
 * from the phonon Green's function blocks of the paper's 6-D tensor
 *   Dfull [nqz][nw][na][nb+1][3][3]: slot 0 = D_aa, slot 1+n = D_{a, nbr[a,n]}.
 * D_ba is Dfull[.., b, 1+m] with nbr[b,m] = a (the table must be symmetric).
 * Output Dc [nqz][nw][na][nb][3][3].  Returns 6 if some pair has no reverse slot.
 */
int oracle_combine_d(const int64_t* dims, const double* Dfull, const int32_t* nbr, double* Dc) {
    odims d;
    int rc = read_dims(dims, &d);
    if (rc) return rc;
    if (!Dfull || !nbr || !Dc) return 1;
    if ((rc = check_nbr(&d, nbr))) return rc;
    const int64_t S = d.nb + 1;
    for (int64_t a = 0; a < d.na; ++a)
        for (int64_t n = 0; n < d.nb; ++n) {
            const int64_t b = nbr[a * d.nb + n];
            int64_t m = -1;
            for (int64_t t = 0; t < d.nb; ++t)
                if (nbr[b * d.nb + t] == a) { m = t; break; }
            if (m < 0) return 6;
            for (int64_t q = 0; q < d.nqz; ++q)
                for (int64_t w = 0; w < d.nw; ++w)
                    for (int x = 0; x < 9; ++x) {
                        const int64_t base = (q * d.nw + w) * d.na;
                        const double* Dba = Dfull + 2 * (((base + b) * S + 1 + m) * 9 + x);
                        const double* Dbb = Dfull + 2 * (((base + b) * S + 0) * 9 + x);
                        const double* Daa = Dfull + 2 * (((base + a) * S + 0) * 9 + x);
                        const double* Dab = Dfull + 2 * (((base + a) * S + 1 + n) * 9 + x);
                        double* o = Dc + 2 * ((((base + a) * d.nb) + n) * 9 + x);
                        for (int p = 0; p < 2; ++p) o[p] = ((Dba[p] - Dbb[p]) - Daa[p]) + Dab[p];
                    }
        }
    return 0;
}

/*
 * Phonon scattering self-energy (Eq. 4 of the paper, "Current State of the
 * Art"), for the Nb off-diagonal blocks (a, b = nbr[a,n]) the paper keeps,
 * where the sum over l reduces to l = b:
 *
 *   Pi[q, w-1, a, n, i, j] = beta * sum_{k=0}^{Nkz-1} sum_{E: 0 <= E+w < NE}
 *       tr( A[a,n,i]^H . Gs[(k+q) mod Nkz, E+w, a, 0] . A[a,n,j] . Go[k, E, nbr[a,n], 0] )
 *
 * with grad_i H_ba = A[a,n,i]^H and grad_j H_ab = A[a,n,j] (H Hermitian), Gs
 * the electron Green's function of the same component as Pi (its block at
 * atom a, shifted by +qz and +w) and Go the opposite component (its block at
 * the neighbour b, unshifted); beta carries the prefactor -i and the energy
 * quadrature weight.  Each term is formed as written: X = A_i^H . Gs,
 * Y = X . A_j, then the trace of Y . Go.
 *
 * Output Pi [nqz][nw][na][nb][3][3] (the layout of D).
 */

/* out = X^H . Y   (N x N complex) */
static void mat_mul_adj_left(int64_t N, const double* X, const double* Y, cplx* out) {
    for (int64_t r = 0; r < N; ++r)
        for (int64_t c = 0; c < N; ++c) {
            cplx s = { 0.0, 0.0 };
            for (int64_t t = 0; t < N; ++t) s = c_add(s, c_mul(c_conj(c_at(X, t * N + r)), c_at(Y, t * N + c)));
            out[r * N + c] = s;
        }
}

/* One 3x3 output block Pi[q, wi, a, n] (wi = w - 1), written to out as 9 complex. */
static void pi_block(const odims* d, const double* Gs, const double* Go, const double* A, const int32_t* nbr,
                     cplx beta, int64_t q, int64_t wi, int64_t a, int64_t n, cplx* X, cplx* Y, double* out) {
    const int64_t N = d->norb, w = wi + 1;
    const int64_t b = nbr[a * d->nb + n];
    cplx acc[9];
    for (int x = 0; x < 9; ++x) { acc[x].re = 0.0; acc[x].im = 0.0; }
    for (int64_t k = 0; k < d->nkz; ++k) {
        const int64_t ks = (k + q) % d->nkz;
        for (int64_t e = 0; e < d->ne; ++e) {
            const int64_t es = e + w;
            if (es >= d->ne) continue;
            const double* Gsa = Gs + 2 * off_G(d, ks, es, a);
            const double* Gob = Go + 2 * off_G(d, k, e, b);
            for (int i = 0; i < 3; ++i) {
                mat_mul_adj_left(N, A + 2 * off_A(d, a, n, i), Gsa, X);
                for (int j = 0; j < 3; ++j) {
                    const double* Aj = A + 2 * off_A(d, a, n, j);
                    for (int64_t r = 0; r < N; ++r)
                        for (int64_t c = 0; c < N; ++c) {
                            cplx s = { 0.0, 0.0 };
                            for (int64_t t = 0; t < N; ++t) s = c_add(s, c_mul(X[r * N + t], c_at(Aj, t * N + c)));
                            Y[r * N + c] = s;
                        }
                    cplx tr = { 0.0, 0.0 };
                    for (int64_t r = 0; r < N; ++r)
                        for (int64_t u = 0; u < N; ++u) tr = c_add(tr, c_mul(Y[r * N + u], c_at(Gob, u * N + r)));
                    acc[i * 3 + j] = c_add(acc[i * 3 + j], tr);
                }
            }
        }
    }
    for (int x = 0; x < 9; ++x) {
        const cplx v = c_mul(beta, acc[x]);
        out[2 * x] = v.re;
        out[2 * x + 1] = v.im;
    }
}

/* Pi at a list of output blocks pts[p] = (q, w-1, a, n); out is [npts][3][3]. */
int oracle_pse_points(const int64_t* dims, const double* Gs, const double* Go, const double* A,
                      const int32_t* nbr, double beta_re, double beta_im, int64_t npts, const int64_t* pts,
                      double* out) {
    odims d;
    int rc = read_dims(dims, &d);
    if (rc) return rc;
    if (!Gs || !Go || !A || !nbr || (npts > 0 && (!pts || !out))) return 1;
    if ((rc = check_nbr(&d, nbr))) return rc;
    for (int64_t p = 0; p < npts; ++p)
        if (pts[4 * p] < 0 || pts[4 * p] >= d.nqz || pts[4 * p + 1] < 0 || pts[4 * p + 1] >= d.nw ||
            pts[4 * p + 2] < 0 || pts[4 * p + 2] >= d.na || pts[4 * p + 3] < 0 || pts[4 * p + 3] >= d.nb)
            return 2;
    const cplx beta = { beta_re, beta_im };
    const int64_t NN = d.norb * d.norb;
    int fail = 0;
#pragma omp parallel
    {
        cplx* X = (cplx*)malloc(sizeof(cplx) * NN);
        cplx* Y = (cplx*)malloc(sizeof(cplx) * NN);
        if (!X || !Y) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t p = 0; p < npts; ++p)
                pi_block(&d, Gs, Go, A, nbr, beta, pts[4 * p], pts[4 * p + 1], pts[4 * p + 2], pts[4 * p + 3], X, Y,
                         out + 18 * p);
        }
        free(X);
        free(Y);
    }
    return fail ? 7 : 0;
}

/* Full Pi [nqz][nw][na][nb][3][3]. */
int oracle_pse_forward(const int64_t* dims, const double* Gs, const double* Go, const double* A,
                       const int32_t* nbr, double beta_re, double beta_im, double* Pi) {
    odims d;
    int rc = read_dims(dims, &d);
    if (rc) return rc;
    if (!Gs || !Go || !A || !nbr || !Pi) return 1;
    if ((rc = check_nbr(&d, nbr))) return rc;
    const cplx beta = { beta_re, beta_im };
    const int64_t NN = d.norb * d.norb;
    const int64_t nblk = d.nqz * d.nw * d.na * d.nb;
    int fail = 0;
#pragma omp parallel
    {
        cplx* X = (cplx*)malloc(sizeof(cplx) * NN);
        cplx* Y = (cplx*)malloc(sizeof(cplx) * NN);
        if (!X || !Y) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t x = 0; x < nblk; ++x) {
                const int64_t n = x % d.nb, a = (x / d.nb) % d.na, wi = (x / (d.nb * d.na)) % d.nw,
                              q = x / (d.nb * d.na * d.nw);
                pi_block(&d, Gs, Go, A, nbr, beta, q, wi, a, n, X, Y, Pi + 18 * x);
            }
        }
        free(X);
        free(Y);
    }
    return fail ? 7 : 0;
}
