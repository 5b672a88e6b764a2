/*
 * sse.h -- C ABI of libsse, the MI355X (gfx950) implementation of the
 * electron-phonon scattering self-energy of Ziogas et al., "A Data-Centric
 * Approach to Extreme-Scale Ab initio Dissipative Quantum Transport
 * Simulations" (SC'19).
 *
 * The operation (Eq. 3, Sec. "Current State of the Art"), for one of the
 * lesser / greater components (the same superscript on G and D):
 *
 *   Sigma[k,E,a] = alpha * sum_{q=0}^{Nqz-1} sum_{w=1}^{Nw} sum_{s=+1,-1} [0 <= E - s*w < NE]
 *                  * sum_{n=0}^{NB-1} sum_{i,j=0}^{2}
 *                    D[q, w-1, a, n, i, j] * dH[a,n,i] . G[(k-q) mod Nkz, E - s*w, nbr[a,n], 0] . dH[a,n,j]^H
 *
 * - Only the diagonal Norb x Norb block of Sigma per atom is formed (the
 *   paper keeps only the diagonal blocks of the electron SSE).
 * - dH[a,n,i] = grad_i H for the pair (a, b = nbr[a,n]); grad_j H_ba is taken
 *   as dH[a,n,j]^H (H is Hermitian).
 * - D[q, w-1, a, n, :, :] is the phonon coefficient of the pair (a, nbr[a,n])
 *   with the bracket (D_ba - D_bb - D_aa + D_ab) already formed; the phonon
 *   frequency w*dE sits on the electron energy grid, w = 1..Nw.
 * - Both energy branches E -/+ w use the same D; points outside the energy
 *   grid contribute zero; the momentum grids coincide (Nqz = Nkz) and are
 *   periodic, so kz - qz wraps around.
 * - alpha carries the prefactor i of Eq. 3 and any quadrature weight of the
 *   frequency integral the caller did not fold into D.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - All tensor pointers are HIP device pointers to row-major, contiguous
 *   arrays.  "complex" means interleaved (re, im) doubles, i.e. the memory
 *   of a complex128 tensor.  n3d is fixed at 3.
 * - Shapes:
 *     G       [nkz][ne][na][g_slots][norb][norb] complex; only slot 0 is read
 *     D       [nqz][nw][na][nb][3][3]            complex
 *     dH      [na][nb][3][norb][norb]            complex
 *     nbr     [na][nb]                           int32, entries in [0, na)
 *     Sigma   [nkz][ne][na][norb][norb]          complex (output)
 *     dSigma  like Sigma; dG like G; dD like D; ddH like dH
 * - Ownership: the caller allocates and frees every buffer, including the
 *   workspace (size from sse_workspace_bytes).  The library keeps no device
 *   allocations and does no host<->device copies, except the one status word
 *   that sse_check_nbr and sse_combine_d read back.
 * - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *   stream).  Outputs are overwritten, never accumulated.  Inputs are only
 *   read.  Calls that use distinct outputs and workspaces may run
 *   concurrently.
 * - Status codes (no exceptions cross this boundary; on an argument error --
 *   every code but SSE_ERR_HIP -- no kernel has been launched and no output has
 *   been touched; an SSE_ERR_HIP from a call that launches several kernels may
 *   leave its outputs partly written):
 *     SSE_OK 0, SSE_ERR_NULL 1 (required pointer is NULL), SSE_ERR_DIMS 2
 *     (a dim <= 0, nqz != nkz, g_slots < 1, a size beyond the supported
 *     limits, or an element count that overflows int64), SSE_ERR_WORKSPACE 3,
 *     SSE_ERR_PRECISION 4, SSE_ERR_HIP 5 (the message carries
 *     hipGetErrorString), SSE_ERR_NBR 6 (sse_check_nbr found an entry outside
 *     [0, na), or sse_combine_d found the table not symmetric).
 *   sse_last_error() returns a thread-local description of the last failure.
 * - Kernels never read outside their inputs: a neighbour entry outside
 *   [0, na) contributes zero (validate tables with sse_check_nbr).
 */
#ifndef SSE_H
#define SSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSE_ABI_VERSION 6

typedef struct sse_dims {
    int64_t nkz;     /* electron momentum points kz (periodic grid)              */
    int64_t ne;      /* energy points                                            */
    int64_t nqz;     /* phonon momentum points qz; must equal nkz                */
    int64_t nw;      /* phonon frequencies w = 1..nw (units of the energy step)  */
    int64_t na;      /* atoms                                                    */
    int64_t nb;      /* neighbour slots per atom                                 */
    int64_t norb;    /* orbitals per atom (block size)                           */
    int64_t g_slots; /* size of G's block axis (slot 0 = diagonal block G_aa)    */
} sse_dims;

enum sse_precision {
    SSE_FP64 = 0,    /* fp64 products on matrix cores, fp64 reduction                  */
    SSE_FP32 = 1,    /* operands of the dense products rounded to fp32 after the fp64
                        gather, fp32 matrix cores, each 36-term K chunk accumulated in
                        fp32 then added in fp64; fp64 (qz, w, +/-) reduction            */
    SSE_BF16X2 = 2,  /* every operand of the dense product split into bfloat16 hi + lo
                        (hi = bf16(x), lo = bf16(x - hi); bf16 has the exponent range of
                        fp32, so no scaling), the four partial products on the bf16
                        matrix cores, fp32 accumulation per K chunk, fp64 (qz, w, +/-)
                        reduction.  About 16 significant bits per operand: expect
                        relative errors near 1e-5                                        */
    SSE_BF16X3 = 3,  /* three-term bfloat16 split (24 significant bits); declared for
                        the interface, not built: every call returns SSE_ERR_PRECISION    */
    SSE_FP16X2 = 4,  /* half precision with compensation (Sec. "Mixed-Precision
                        Computation"): D, grad H and the left products normalised
                        by powers of two (per atom; per K chunk and source energy),
                        every operand of the dense product split into fp16 hi + lo,
                        the four partial products on the fp16 matrix cores, each K
                        chunk accumulated in fp32, unscaled and added in fp64; fp64
                        gather and (qz, w, +/-) reduction                           */
    SSE_FP16 = 5,    /* the paper's half-precision scheme as it describes it (Sec.
                        "Mixed-Precision Computation"): the normalisation of
                        SSE_FP16X2 with one fp16 term per operand (no lo parts),
                        fp32 accumulation per K chunk, fp64 reduction.  11
                        significant bits per operand: expect relative errors near
                        1e-4.  A comparison form: it runs the SSE_FP16X2 kernel with
                        the lo terms dropped, not a kernel tuned for one term.  One
                        coefficient table only (sse_forward, or the other entry
                        points with Dm == Dp), on the matrix-core shapes; otherwise
                        SSE_ERR_PRECISION                                           */
    SSE_FP16_UNSCALED = 6 /* SSE_FP16 without the power-of-two factors: every operand
                        rounded to fp16 as it is, magnitudes beyond the fp16 range
                        clamped to 65504, values below it kept as fp16 subnormals
                        or zero.  The paper's comparison for its normalisation
                        (Sec. "Mixed-Precision Convergence"); same limits as
                        SSE_FP16                                                    */
};

enum sse_status {
    SSE_OK = 0,
    SSE_ERR_NULL = 1,
    SSE_ERR_DIMS = 2,
    SSE_ERR_WORKSPACE = 3,
    SSE_ERR_PRECISION = 4,
    SSE_ERR_HIP = 5,
    SSE_ERR_NBR = 6
};

/* ABI version of the loaded library (SSE_ABI_VERSION of its build). */
int sse_abi_version(void);

/* Thread-local text of the last error (empty string if none). */
const char* sse_last_error(void);

/*
 * Bytes of workspace a call needs.  op = 0 for sse_forward with the given
 * precision, 1 for sse_backward and sse_backward_signed with every gradient
 * (enough for either; a call without ddH needs less, see sse_backward), 2 for
 * sse_combine_d (precision ignored for 1 and 2).
 */
int sse_workspace_bytes(const sse_dims* dims, int precision, int op, size_t* bytes);

/*
 * Effective flops of one sse_forward call (one component), the paper's
 * computation-model count for the regrouped form: one left product
 * grad_i H . G per (kz', E', a, n, i) plus one product per
 * (kz, E, a, n, i, qz, w, +/-), at 8 Norb^3 flops per complex product
 * (Sec. "Computation Model"):
 *   f_eff = 8 Norb^3 * 3 * NB * Na * Nkz * NE * (2 Nqz Nw + 1).
 */
int sse_effective_flops(const sse_dims* dims, double* f_eff);

/*
 * Sigma = the operation above (Eq. 3).  precision is an sse_precision value;
 * every form reads the same fp64 inputs, gathers them in fp64 and reduces
 * over (qz, w, +/-) in fp64.  Sigma is fully overwritten.  The matrix-core
 * shapes (norb, nkz = nqz, nw, nb) are (10, 7, 10, 4), (10, 7, 10, 3) and
 * (4, 3, 2, 4) for every precision, and (12, 7, 10, 4) for SSE_FP64 and
 * SSE_FP32; other shapes take SSE_FP64 only, on a direct vector-ALU kernel
 * (any other precision: SSE_ERR_PRECISION).
 */
int sse_forward(const sse_dims* dims, const double* G, const double* D, const double* dH,
                const int32_t* nbr, double alpha_re, double alpha_im, int precision,
                double* Sigma, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Sigma of Eq. 3 with its frequency integral taken over both signs of w on a
 * grid of Nw positive frequencies w_m = m (m = 1..Nw, energy steps):
 *
 *   Sigma[k,E,a] = alpha * sum_q sum_{m=1}^{Nw} sum_n sum_{i,j}
 *                  ( [E-m >= 0] Dp[q,m-1,a,n,i,j] grad_iH . G[(k-q) mod Nkz, E-m, nbr[a,n], 0] . grad_jH^H
 *                  + [E+m < NE] Dm[q,m-1,a,n,i,j] grad_iH . G[(k-q) mod Nkz, E+m, nbr[a,n], 0] . grad_jH^H )
 *
 * Dp holds the coefficients at +w_m (the terms with G at E - w) and Dm those at
 * -w_m (G at E + w), both in D's layout [nqz][nw][na][nb][3][3]; how Dm is
 * obtained (for instance from a lesser/greater symmetry of D) is the caller's.
 * With Dm == Dp (the same pointer) this is sse_forward, in one pass.
 * Otherwise the matrix-core shapes run one pass per table (the E - w terms
 * write Sigma, the E + w terms add to it: twice the work of sse_forward); the
 * other shapes take both tables in one fp64 pass.  Other arguments, layouts,
 * precisions, workspace and errors as for sse_forward; Sigma must not overlap
 * an input.
 */
int sse_forward_signed(const sse_dims* dims, const double* G, const double* Dp, const double* Dm,
                       const double* dH, const int32_t* nbr, double alpha_re, double alpha_im,
                       int precision, double* Sigma, void* workspace, size_t workspace_bytes,
                       void* stream);

/*
 * The full input contract of Eq. 3: one coefficient table per sign of the
 * frequency as in sse_forward_signed (Dm == Dp: the one-table form of
 * sse_forward) and the right factor grad_j H_ba as stored blocks:
 *
 *   Sigma[k,E,a] = alpha * sum_q sum_{m=1}^{Nw} sum_n sum_{i,j}
 *                  ( [E-m >= 0] Dp[q,m-1,a,n,i,j] dH[a,n,i] . G[(k-q) mod Nkz, E-m, nbr[a,n], 0] . dHba[a,n,j]
 *                  + [E+m < NE] Dm[q,m-1,a,n,i,j] dH[a,n,i] . G[(k-q) mod Nkz, E+m, nbr[a,n], 0] . dHba[a,n,j] )
 *
 * dHba [na][nb][3][norb][norb] complex holds grad_j H_ba for the pair (a, b =
 * nbr[a,n]) (the layout of dH); NULL means the Hermitian reading dHba[a,n,j] =
 * dH[a,n,j]^H, which makes this call sse_forward_signed.  Every precision runs
 * on the matrix-core shapes with norb 10 or 4 (the fp64 kernel then works on
 * energy blocks of four, whose LDS holds the second table); at norb 12 and on
 * other shapes a stored dHba takes fp64 only, on the direct kernel.  Other
 * arguments, layouts, workspace and errors as for sse_forward_signed.
 */
int sse_forward_ex(const sse_dims* dims, const double* G, const double* Dp, const double* Dm, const double* dH,
                   const double* dHba, const int32_t* nbr, double alpha_re, double alpha_im, int precision,
                   double* Sigma, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Adjoint of sse_forward (fp64) for a real scalar L, given dSigma = dL/dSigma
 * in PyTorch's convention for complex gradients (dL/dRe z + i dL/dIm z).
 * Writes dL/dG (slots >= 1 set to zero), dL/dD and dL/d(dH); any of the three
 * output pointers may be NULL to skip that gradient.  Per valid term with
 * d = D[q,w-1,a,n,i,j], A_i = dH[a,n,i], B = G[k',E',b,0], g = dSigma[k,E,a]:
 *   dG[k',E',b,0]     += conj(alpha d) A_i^H g A_j
 *   dD[q,w-1,a,n,i,j] += conj(alpha) sum_{r,c} conj((A_i B A_j^H)[r,c]) g[r,c]
 *   ddH[a,n,i]        += conj(alpha d) g A_j B^H
 *   ddH[a,n,j]        += alpha d g^H A_i B
 * Shifted G blocks are re-gathered, not stored.  The workspace
 * (sse_workspace_bytes(dims, 0, 1) bytes suffice for every call) holds the
 * reverse neighbour adjacency and the atoms' dispatch order (4 * (4 na + 1 +
 * na * nb) bytes, rounded up to
 * 256) and, if ddH is wanted, S shares of every edge's dL/d(dH)
 * (16 * S * na * nb * 3 * norb^2 bytes, rounded up to 256), added in share
 * order, so results are bitwise reproducible: S = ceil(ne / 32) (one per range
 * of 32 energies) on the matrix-core shape (norb = 10, nkz = nqz = 7, nw = 10),
 * S = nkz (one per momentum) otherwise and in sse_backward_signed.  If dD is
 * wanted on the shapes of the matrix-core phonon kernel (norb = 10, nkz = nqz
 * = 7, nw = 10, nb = 4 or 3), it also holds a copy of dSigma with the atom
 * axis first (16 * na * nkz * ne * norb^2 bytes, the size of dSigma), from
 * which the dD kernel reads its shifted blocks of both energy branches (the
 * same sums in the same order as from dSigma itself; sse_backward_signed
 * reads one branch per launch from dSigma in place and needs no copy).  A smaller workspace than this call uses is
 * refused with SSE_ERR_WORKSPACE.  An entry of nbr outside [0, na) has no
 * terms: its ddH block is zero.
 */
int sse_backward(const sse_dims* dims, const double* G, const double* D, const double* dH,
                 const int32_t* nbr, double alpha_re, double alpha_im, const double* dSigma,
                 double* dG, double* dD, double* ddH, void* workspace, size_t workspace_bytes,
                 void* stream);

/*
 * Adjoint of sse_forward_signed (fp64): as sse_backward, with the gradients of
 * both coefficient tables.  The terms with G at E - m read Dp and feed dDp, the
 * terms with G at E + m read Dm and feed dDm; per valid term with d the
 * coefficient of its table the formulas of sse_backward apply.  dG, dDp, dDm
 * and ddH may each be NULL to skip it.  Workspace as for sse_backward.
 */
int sse_backward_signed(const sse_dims* dims, const double* G, const double* Dp, const double* Dm,
                        const double* dH, const int32_t* nbr, double alpha_re, double alpha_im,
                        const double* dSigma, double* dG, double* dDp, double* dDm, double* ddH,
                        void* workspace, size_t workspace_bytes, void* stream);

/*
 * sse_backward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same results bit for bit, with the workspace in a device array that is part
 * of the library (sse_noalloc_scratch_bytes() bytes, 64 MiB, held by every GPU
 * the library runs on until the process ends) instead of a caller-provided
 * buffer.  Calls no hipMalloc, hipFree or allocating routine.  Dims whose
 * workspace for this call exceeds the array are rejected with
 * SSE_ERR_WORKSPACE before anything is launched: the reverse adjacency takes
 * 4 * (4 Na + 1 + Na * Nb) bytes (rounded up to 256), and with ddH the d(dH)
 * shares 16 * S * Na * Nb * 3 * Norb^2 more, S = ceil(NE / 32)
 * on the matrix-core shape (Norb = 10, Nkz = Nqz = 7, Nw = 10), S = Nkz otherwise
 * (at Nkz = 7, Norb = 10, Nb = 4, NE <= 224: about 500 atoms with ddH, about
 * 2.1 million without it).  dD reads dSigma in place (no atom-major copy:
 * slower than sse_backward's, the same sums).  Every call on one GPU uses that GPU's
 * array (the current device's): calls that overlap on one GPU race.  The
 * kernels rewrite every part of the array they read, so no clearing is needed
 * between calls.  Other arguments and errors as for sse_backward.
 */
int sse_backward_noalloc(const sse_dims* dims, const double* G, const double* D, const double* dH,
                         const int32_t* nbr, double alpha_re, double alpha_im, const double* dSigma,
                         double* dG, double* dD, double* ddH, void* stream);

/* Size in bytes of the device array behind sse_backward_noalloc. */
size_t sse_noalloc_scratch_bytes(void);

/*
 * Coefficients of the absorption branch of Eq. 3 (the frequency -w of its
 * integral over signed frequencies, the Dm argument of sse_forward_signed and
 * sse_forward_ex) from the combined table of the opposite component:
 *   Dm[q,w,a,n,i,j] = Dopp[(nqz - q) mod nqz, w, a, n, j, i].
 * The paper gives no relation for D(-w); this one holds for real displacement
 * fields, D<_ab(q, -w) = D>_ba(-q, w) (and with < and > exchanged), and the
 * bracket D_ba - D_bb - D_aa + D_ab of Eq. 3 is symmetric in a <-> b.  So for
 * Sigma< pass Dp = D< and Dm = sse_absorption_d(D>), for Sigma> Dp = D> and
 * Dm = sse_absorption_d(D<).  Dopp and Dm are [nqz][nw][na][nb][3][3] complex;
 * a permutation of entries, bit for bit.  Dm must not overlap Dopp
 * (SSE_ERR_DIMS).  No workspace.
 */
int sse_absorption_d(const sse_dims* dims, const double* Dopp, double* Dm, void* stream);

/*
 * The bracket of Eq. 3 for every neighbour slot, the step that prepares D:
 *   D[q,w,a,n,:,:] = Dfull[q,w,b,1+m] - Dfull[q,w,b,0] - Dfull[q,w,a,0] + Dfull[q,w,a,1+n]
 * (= D_ba - D_bb - D_aa + D_ab) with b = nbr[a,n] and m the slot with
 * nbr[b,m] = a.  Dfull [nqz][nw][na][nb+1][3][3] complex holds the phonon
 * Green's function blocks the paper's SSE reads: slot 0 the diagonal block
 * D_aa, slot 1+n the block coupling a to nbr[a,n].  Output D
 * [nqz][nw][na][nb][3][3], the D argument of sse_forward.  The table must be
 * symmetric (a in nbr[b] whenever b in nbr[a]); this is checked first,
 * synchronously on `stream` (SSE_ERR_NBR, nothing written, if it fails).
 * Workspace: sse_workspace_bytes(dims, 0, 2).
 */
int sse_combine_d(const sse_dims* dims, const double* Dfull, const int32_t* nbr, double* D, void* workspace,
                  size_t workspace_bytes, void* stream);

/*
 * Phonon scattering self-energy (Eq. 4, Sec. "Current State of the Art") for
 * the NB off-diagonal blocks per atom that the paper keeps, (a, b = nbr[a,n]),
 * where the sum over l reduces to l = b:
 *
 *   Pi[q, w-1, a, n, i, j] = beta * sum_{k=0}^{Nkz-1} sum_{E : 0 <= E+w < NE}
 *       tr( dH[a,n,i]^H . Gs[(k+q) mod Nkz, E+w, a, 0] . dH[a,n,j] . Go[k, E, nbr[a,n], 0] )
 *
 * grad_i H_ba = dH[a,n,i]^H and grad_j H_ab = dH[a,n,j] (H is Hermitian).  Gs
 * is the electron Green's function of the same component as Pi (G< for Pi<),
 * Go the opposite one (G> for Pi<), both laid out like G (slot 0 read).  beta
 * carries the prefactor -i of Eq. 4 and the energy quadrature weight.  The
 * phonon frequency w sits on the electron energy grid, w = 1..Nw; the momentum
 * grids coincide (Nqz = Nkz) and kz + qz wraps around.
 * Output Pi [nqz][nw][na][nb][3][3] complex (the layout of D), fully
 * overwritten.  fp64 throughout; no workspace.  Gs and Go may alias.
 * Errors as for sse_forward (SSE_ERR_DIMS also when no kernel covers the
 * shape: norb^2 > 640 or nqz * nw > 512 outside the matrix-core shape).
 */
int sse_phonon_forward(const sse_dims* dims, const double* Gs, const double* Go, const double* dH,
                       const int32_t* nbr, double beta_re, double beta_im, double* Pi, void* stream);

/*
 * Synchronous check of a neighbour table: returns SSE_OK if every entry lies
 * in [0, na), SSE_ERR_NBR otherwise.  Needs sse_workspace_bytes(dims, 0, 0)
 * bytes of workspace, at least 4; copies one int32 back to the host and waits
 * on `stream`.
 */
int sse_check_nbr(const sse_dims* dims, const int32_t* nbr, void* workspace, size_t workspace_bytes,
                  void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SSE_H */
