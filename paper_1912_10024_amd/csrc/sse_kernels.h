// Launch entry points of the kernels behind the C ABI.
#pragma once

#include "sse_common.h"

namespace sse {

// Energy branches of Eq. 3 on a grid of positive frequencies w: the terms with
// G at E - w (coefficient at +w) and those with G at E + w (coefficient at -w)
constexpr int kBranchMinus = 1;  // terms with G at E - w
constexpr int kBranchPlus = 2;   // terms with G at E + w
constexpr int kAccumulate = 4;   // Sigma += result instead of Sigma = result

// direct term-by-term fp64 forward (any shape with norb^2 <= 1024); the terms
// with G at E - w read Dp, those with G at E + w read Dm (Dm == Dp: the
// one-table form of sse_forward); B = stored grad_j H_ba blocks (layout of A),
// or nullptr for A^H
bool generic_supported(const Dims& d);
hipError_t launch_fwd_generic(const Dims& d, const double* G, const double* Dp, const double* Dm, const double* A,
                              const double* B, const int32_t* nbr, cd alpha, double* S, hipStream_t stream);

// matrix-core forward (fp64 or fp32 operands; the split 16-bit forms go to
// launch_fwd_h16) for the shapes it is
// instantiated for; flags selects the energy branches (kBranchMinus,
// kBranchPlus) and whether the result is added to Sigma (kAccumulate)
// B: stored grad_j H_ba blocks (layout of A) as the right factor, or nullptr for A^H
bool fwd_mfma_specialised(const Dims& d);
// whether the matrix-core forward takes this precision (and a stored grad H_ba) at these dims
bool fwd_mfma_supports(const Dims& d, int precision, bool hba);
hipError_t launch_fwd_mfma(const Dims& d, int precision, const double* G, const double* D, const double* A,
                           const double* B, const int32_t* nbr, cd alpha, double* S, hipStream_t stream,
                           int flags = kBranchMinus | kBranchPlus);

// matrix-core forward with split 16-bit operands (SSE_FP16X2, SSE_BF16X2, and the
// single-term SSE_FP16 and SSE_FP16_UNSCALED with the flags of the one-table form
// only) for the shapes of fwd_mfma_specialised; B and flags as for launch_fwd_mfma
hipError_t launch_fwd_h16(const Dims& d, int precision, const double* G, const double* D, const double* A,
                          const double* B, const int32_t* nbr, cd alpha, double* S, hipStream_t stream, int flags);

// adjoint (fp64): reverse adjacency in the workspace, then dG/d gradH per neighbour atom and dD.
// signed_form: the terms with G at E - w read Dp and feed dDp, those at E + w
// read Dm and feed dDm; otherwise Dp is the one table and dDp its gradient (Dm,
// dDm unused).
size_t bwd_workspace_bytes(const Dims& d);  // enough for either form, with every gradient
// what one call uses: the reverse adjacency, plus the d gradH shares if that
// gradient is asked for, plus the atom-major copy of g if the D gradient of the
// one-table form is asked for with copy_g (on the dims that take it: pse_atom_major_ok)
size_t bwd_workspace_bytes_for(const Dims& d, bool signed_form, bool with_dh, bool with_dd = false,
                               bool copy_g = false);
bool bwd_supported(const Dims& d);
// dG and d gradH of the one-table form on the matrix cores (Norb = 10, Nkz = Nqz = 7,
// Nw = 10): one workgroup per (neighbour atom, range of energies), one d gradH
// share per range (bwd_mfma_shares of them) in dApart
bool bwd_mfma_specialised(const Dims& d);
int64_t bwd_mfma_shares(const Dims& d);
hipError_t bwd_mfma_prepare();
hipError_t launch_bwd_mfma(const Dims& d, const double* G, const double* D, const double* A, const double* gS, cd calpha,
                           const int32_t* offset, const int32_t* edges, const int32_t* order, double* dG,
                           double* dApart, hipStream_t stream);
hipError_t launch_bwd(const Dims& d, const double* G, const double* Dp, const double* Dm, const double* A,
                      const int32_t* nbr, cd alpha, const double* gS, double* dG, double* dDp, double* dDm, double* dA,
                      void* ws, hipStream_t stream, bool signed_form, bool copy_g);

// absorption-branch coefficients: Dm[q,w,a,n,i,j] = Dopp[(-q) mod nqz, w, a, n, j, i]
hipError_t launch_absorption_d(const Dims& d, const double* Dopp, double* Dm, hipStream_t stream);

// Eq. 3 bracket from the full phonon blocks (symmetric neighbour table)
size_t combine_workspace_bytes(const Dims& d);
hipError_t launch_reverse_slots(const Dims& d, const int32_t* nbr, void* ws, hipStream_t stream);
hipError_t launch_combine_d(const Dims& d, const double* Dfull, const int32_t* nbr, double* Dc, void* ws,
                            hipStream_t stream);

// phonon self-energy (Eq. 4, off-diagonal blocks): matrix-core kernel for the shape it is
// instantiated for, a vector-ALU kernel for every other shape that fits
bool pse_mfma_specialised(const Dims& d);
bool pse_generic_supported(const Dims& d);
hipError_t launch_pse(const Dims& d, const double* Gs, const double* Go, const double* A, const int32_t* nbr, cd beta,
                      double* Pi, hipStream_t stream);
// the D gradient of the adjoint on the same matrix-core kernel (shapes with
// pse_mfma_specialised); branches: 1 the terms with G at E - w (coefficients at
// +w), 2 those with G at E + w (at -w), 3 both (the one-table form).  gT: the
// atom-major copy of gS written by pse_atom_major_g (read in its place), or NULL
hipError_t launch_dd_mfma(const Dims& d, const double* G, const double* A, const int32_t* nbr, const double* gS,
                          const double* gT, cd calpha, double* dD, hipStream_t stream, int branches = 3);
// the atom-major copy of g for the D gradient: whether these dims take it, its
// bytes (0 when they do not), and the copy itself (every byte written)
bool pse_atom_major_ok(const Dims& d);
size_t pse_atom_major_bytes(const Dims& d);
hipError_t pse_atom_major_g(const Dims& d, const double* g, double* gT, hipStream_t stream);

// sse_backward with copy_g = true; false: the D gradient reads g in the caller's
// layout and the workspace holds no copy of it (sse_backward_noalloc)
int backward_one_table(const sse_dims* dims, const double* G, const double* D, const double* dH, const int32_t* nbr,
                       double alpha_re, double alpha_im, const double* dSigma, double* dG, double* dD, double* ddH,
                       void* workspace, size_t workspace_bytes, void* stream, bool copy_g);

// sets the thread-local text that sse_last_error returns; returns code
int set_error(int code, const char* fmt, ...);

// neighbour-table range check: sets *flag (device int) to 1 if any entry is outside [0, na)
hipError_t launch_check_nbr(const Dims& d, const int32_t* nbr, int* flag, hipStream_t stream);

}  // namespace sse
