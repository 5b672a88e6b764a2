// C ABI of libsse: argument validation, workspace sizing and kernel dispatch.
// Every check happens before any HIP call, so an invalid call launches nothing
// and leaves every output untouched.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "sse_kernels.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int ok() {
    g_err[0] = '\0';
    return SSE_OK;
}

}  // namespace

namespace sse {
int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}
}  // namespace sse

namespace {

// a*b with overflow detection for non-negative operands
bool mul_ok(int64_t a, int64_t b, int64_t* out) {
    if (a < 0 || b < 0) return false;
    if (a != 0 && b > INT64_MAX / a) return false;
    *out = a * b;
    return true;
}

bool count_ok(std::initializer_list<int64_t> xs) {
    int64_t acc = 2;  // doubles per complex
    for (int64_t x : xs)
        if (!mul_ok(acc, x, &acc)) return false;
    return true;
}

constexpr int64_t kMaxNorb = 32;

int check_dims(const sse_dims* d) {
    if (!d) return fail(SSE_ERR_NULL, "dims is NULL");
    if (d->nkz <= 0 || d->ne <= 0 || d->nqz <= 0 || d->nw <= 0 || d->na <= 0 || d->nb <= 0 || d->norb <= 0 ||
        d->g_slots <= 0)
        return fail(SSE_ERR_DIMS, "every dim must be positive (nkz=%lld ne=%lld nqz=%lld nw=%lld na=%lld nb=%lld norb=%lld g_slots=%lld)",
                    (long long)d->nkz, (long long)d->ne, (long long)d->nqz, (long long)d->nw, (long long)d->na,
                    (long long)d->nb, (long long)d->norb, (long long)d->g_slots);
    if (d->nqz != d->nkz) return fail(SSE_ERR_DIMS, "nqz (%lld) must equal nkz (%lld)", (long long)d->nqz, (long long)d->nkz);
    if (d->norb > kMaxNorb) return fail(SSE_ERR_DIMS, "norb %lld exceeds the supported maximum %lld", (long long)d->norb, (long long)kMaxNorb);
    if (d->na > INT32_MAX) return fail(SSE_ERR_DIMS, "na %lld does not fit the int32 neighbour table", (long long)d->na);
    if (!count_ok({d->nkz, d->ne, d->na, d->g_slots, d->norb, d->norb}) || !count_ok({d->nqz, d->nw, d->na, d->nb, 9}) ||
        !count_ok({d->na, d->nb, 3, d->norb, d->norb}) || !count_ok({d->nkz, d->ne, d->na, d->norb, d->norb}))
        return fail(SSE_ERR_DIMS, "tensor sizes overflow int64");
    return SSE_OK;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SSE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool precision_known(int p) {
    return p == SSE_FP64 || p == SSE_FP32 || p == SSE_BF16X2 || p == SSE_BF16X3 || p == SSE_FP16X2 || p == SSE_FP16 ||
           p == SSE_FP16_UNSCALED;
}

// precision check of the forward entry points: unknown codes, and the declared
// form without a kernel, are SSE_ERR_PRECISION
int check_precision(int p) {
    if (!precision_known(p)) return fail(SSE_ERR_PRECISION, "unknown precision %d", p);
    if (p == SSE_BF16X3)
        return fail(SSE_ERR_PRECISION,
                    "precision SSE_BF16X3 (three-term bfloat16 split) is not built: its operands take 12 bytes per "
                    "K element, more than the matrix-core kernel's LDS holds; use SSE_FP16X2 or SSE_FP32 for errors "
                    "below 1e-6");
    return SSE_OK;
}

}  // namespace

extern "C" {

int sse_abi_version(void) { return SSE_ABI_VERSION; }

const char* sse_last_error(void) { return g_err; }

int sse_workspace_bytes(const sse_dims* dims, int precision, int backward, size_t* bytes) {
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!bytes) return fail(SSE_ERR_NULL, "bytes is NULL");
    if (backward == 0 && !precision_known(precision)) return fail(SSE_ERR_PRECISION, "unknown precision %d", precision);
    if (backward < 0 || backward > 2) return fail(SSE_ERR_DIMS, "op must be 0 (forward), 1 (backward) or 2 (combine_d)");
    size_t ws = 256;  // status flag of sse_check_nbr
    if (backward == 1) {
        const size_t b = sse::bwd_workspace_bytes(sse::to_dims(*dims));
        if (b > ws) ws = b;
    }
    if (backward == 2) {
        const size_t b = sse::combine_workspace_bytes(sse::to_dims(*dims));
        if (b > ws) ws = b;
    }
    *bytes = ws;
    return ok();
}

int sse_effective_flops(const sse_dims* dims, double* f_eff) {
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!f_eff) return fail(SSE_ERR_NULL, "f_eff is NULL");
    const double n = (double)dims->norb;
    *f_eff = 8.0 * n * n * n * 3.0 * (double)dims->nb * (double)dims->na * (double)dims->nkz * (double)dims->ne *
             (2.0 * (double)dims->nqz * (double)dims->nw + 1.0);
    return ok();
}

}  // extern "C"

namespace {

// Sigma with the terms whose G sits at E - w reading Dp and those at E + w
// reading Dm (the same table for sse_forward), and the right factor dHba (the
// stored grad_j H_ba) or, for NULL, dH^H
int forward_impl(const sse_dims* dims, const double* G, const double* Dp, const double* Dm, const double* dH,
                 const double* dHba, const int32_t* nbr, double alpha_re, double alpha_im, int precision,
                 double* Sigma, void* workspace, size_t workspace_bytes, void* stream) {
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!G || !Dp || !Dm || !dH || !nbr || !Sigma) return fail(SSE_ERR_NULL, "a tensor pointer is NULL");
    if ((rc = check_precision(precision))) return rc;
    if ((precision == SSE_FP16 || precision == SSE_FP16_UNSCALED) && Dm != Dp)
        return fail(SSE_ERR_PRECISION, "precision %d (single-term fp16) is built for one coefficient table (Dm == Dp) only",
                    precision);
    size_t need = 0;
    sse_workspace_bytes(dims, precision, 0, &need);
    if (need > 0 && (workspace == nullptr || workspace_bytes < need))
        return fail(SSE_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    const sse::Dims d = sse::to_dims(*dims);
    const sse::cd alpha{alpha_re, alpha_im};
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if (sse::fwd_mfma_supports(d, precision, dHba != nullptr)) {
        if (Dm == Dp) {
            e = sse::launch_fwd_mfma(d, precision, G, Dp, dH, dHba, nbr, alpha, Sigma, s);
        } else {
            // one GEMM per table: the E - w terms write Sigma, the E + w terms add to it
            e = sse::launch_fwd_mfma(d, precision, G, Dp, dH, dHba, nbr, alpha, Sigma, s, sse::kBranchMinus);
            if (e == hipSuccess)
                e = sse::launch_fwd_mfma(d, precision, G, Dm, dH, dHba, nbr, alpha, Sigma, s,
                                         sse::kBranchPlus | sse::kAccumulate);
        }
    } else {
        if (precision != SSE_FP64)
            return fail(SSE_ERR_PRECISION, "precision %d has no kernel for these dims", precision);
        if (!sse::generic_supported(d)) return fail(SSE_ERR_DIMS, "no kernel for these dims");
        e = sse::launch_fwd_generic(d, G, Dp, Dm, dH, dHba, nbr, alpha, Sigma, s);
    }
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return ok();
}

}  // namespace

extern "C" {

int sse_forward(const sse_dims* dims, const double* G, const double* D, const double* dH, const int32_t* nbr,
                double alpha_re, double alpha_im, int precision, double* Sigma, void* workspace,
                size_t workspace_bytes, void* stream) {
    return forward_impl(dims, G, D, D, dH, nullptr, nbr, alpha_re, alpha_im, precision, Sigma, workspace,
                        workspace_bytes, stream);
}

int sse_forward_signed(const sse_dims* dims, const double* G, const double* Dp, const double* Dm, const double* dH,
                       const int32_t* nbr, double alpha_re, double alpha_im, int precision, double* Sigma,
                       void* workspace, size_t workspace_bytes, void* stream) {
    return forward_impl(dims, G, Dp, Dm, dH, nullptr, nbr, alpha_re, alpha_im, precision, Sigma, workspace,
                        workspace_bytes, stream);
}

int sse_forward_ex(const sse_dims* dims, const double* G, const double* Dp, const double* Dm, const double* dH,
                   const double* dHba, const int32_t* nbr, double alpha_re, double alpha_im, int precision,
                   double* Sigma, void* workspace, size_t workspace_bytes, void* stream) {
    return forward_impl(dims, G, Dp, Dm, dH, dHba, nbr, alpha_re, alpha_im, precision, Sigma, workspace,
                        workspace_bytes, stream);
}

}  // extern "C"

namespace {

int backward_impl(const sse_dims* dims, const double* G, const double* Dp, const double* Dm, const double* dH,
                  const int32_t* nbr, double alpha_re, double alpha_im, const double* dSigma, double* dG,
                  double* dDp, double* dDm, double* ddH, void* workspace, size_t workspace_bytes, void* stream,
                  bool signed_form, bool copy_g) {
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!G || !Dp || !Dm || !dH || !nbr || !dSigma) return fail(SSE_ERR_NULL, "an input pointer is NULL");
    const sse::Dims d = sse::to_dims(*dims);
    if (!sse::bwd_supported(d)) return fail(SSE_ERR_DIMS, "no adjoint kernel for these dims");
    // what this call uses (sse_workspace_bytes covers every gradient of either form)
    const size_t need = sse::bwd_workspace_bytes_for(d, signed_form, ddH != nullptr, dDp || dDm, copy_g);
    if (workspace == nullptr || workspace_bytes < need)
        return fail(SSE_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    if (!dG && !dDp && !dDm && !ddH) return ok();
    hipError_t e = sse::launch_bwd(d, G, Dp, Dm, dH, nbr, sse::cd{alpha_re, alpha_im}, dSigma, dG, dDp, dDm, ddH,
                                   workspace, reinterpret_cast<hipStream_t>(stream), signed_form, copy_g);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return ok();
}

}  // namespace

namespace sse {
int backward_one_table(const sse_dims* dims, const double* G, const double* D, const double* dH, const int32_t* nbr,
                       double alpha_re, double alpha_im, const double* dSigma, double* dG, double* dD, double* ddH,
                       void* workspace, size_t workspace_bytes, void* stream, bool copy_g) {
    return backward_impl(dims, G, D, D, dH, nbr, alpha_re, alpha_im, dSigma, dG, dD, nullptr, ddH, workspace,
                         workspace_bytes, stream, false, copy_g);
}
}  // namespace sse

extern "C" {

int sse_backward(const sse_dims* dims, const double* G, const double* D, const double* dH, const int32_t* nbr,
                 double alpha_re, double alpha_im, const double* dSigma, double* dG, double* dD, double* ddH,
                 void* workspace, size_t workspace_bytes, void* stream) {
    return sse::backward_one_table(dims, G, D, dH, nbr, alpha_re, alpha_im, dSigma, dG, dD, ddH, workspace,
                                   workspace_bytes, stream, true);
}

int sse_backward_signed(const sse_dims* dims, const double* G, const double* Dp, const double* Dm, const double* dH,
                        const int32_t* nbr, double alpha_re, double alpha_im, const double* dSigma, double* dG,
                        double* dDp, double* dDm, double* ddH, void* workspace, size_t workspace_bytes,
                        void* stream) {
    return backward_impl(dims, G, Dp, Dm, dH, nbr, alpha_re, alpha_im, dSigma, dG, dDp, dDm, ddH, workspace,
                         workspace_bytes, stream, true, true);
}

int sse_absorption_d(const sse_dims* dims, const double* Dopp, double* Dm, void* stream) {
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!Dopp || !Dm) return fail(SSE_ERR_NULL, "a tensor pointer is NULL");
    const sse::Dims d = sse::to_dims(*dims);
    const size_t bytes = 16 * (size_t)(d.nqz * d.nw * d.na * d.nb * 9);
    const char* in = reinterpret_cast<const char*>(Dopp);
    const char* out = reinterpret_cast<const char*>(Dm);
    if (in < out + bytes && out < in + bytes) return fail(SSE_ERR_DIMS, "Dm overlaps Dopp");
    hipError_t e = sse::launch_absorption_d(d, Dopp, Dm, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "absorption_d launch");
    return ok();
}

int sse_combine_d(const sse_dims* dims, const double* Dfull, const int32_t* nbr, double* Dc, void* workspace,
                  size_t workspace_bytes, void* stream) {
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!Dfull || !nbr || !Dc) return fail(SSE_ERR_NULL, "a tensor pointer is NULL");
    if (!count_ok({dims->nqz, dims->nw, dims->na, dims->nb + 1, 9})) return fail(SSE_ERR_DIMS, "tensor sizes overflow int64");
    const sse::Dims d = sse::to_dims(*dims);
    const size_t need = sse::combine_workspace_bytes(d);
    if (!workspace || workspace_bytes < need)
        return fail(SSE_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = sse::launch_reverse_slots(d, nbr, workspace, s);
    if (e != hipSuccess) return hip_fail(e, "reverse-slot launch");
    int host_flag = 0;
    e = hipMemcpyAsync(&host_flag, workspace, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "reverse-slot copy");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reverse-slot sync");
    if (host_flag) return fail(SSE_ERR_NBR, "neighbour table is not symmetric or has an entry outside [0, na)");
    e = sse::launch_combine_d(d, Dfull, nbr, Dc, workspace, s);
    if (e != hipSuccess) return hip_fail(e, "combine_d launch");
    return ok();
}

int sse_phonon_forward(const sse_dims* dims, const double* Gs, const double* Go, const double* dH, const int32_t* nbr,
                       double beta_re, double beta_im, double* Pi, void* stream) {
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!Gs || !Go || !dH || !nbr || !Pi) return fail(SSE_ERR_NULL, "a tensor pointer is NULL");
    const sse::Dims d = sse::to_dims(*dims);
    if (!sse::pse_mfma_specialised(d) && !sse::pse_generic_supported(d))
        return fail(SSE_ERR_DIMS, "no phonon self-energy kernel for these dims");
    hipError_t e = sse::launch_pse(d, Gs, Go, dH, nbr, sse::cd{beta_re, beta_im}, Pi, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "phonon forward launch");
    return ok();
}

int sse_check_nbr(const sse_dims* dims, const int32_t* nbr, void* workspace, size_t workspace_bytes, void* stream) {
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!nbr) return fail(SSE_ERR_NULL, "nbr is NULL");
    if (!workspace || workspace_bytes < sizeof(int)) return fail(SSE_ERR_WORKSPACE, "workspace of at least 4 bytes needed");
    const sse::Dims d = sse::to_dims(*dims);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int* flag = reinterpret_cast<int*>(workspace);
    hipError_t e = sse::launch_check_nbr(d, nbr, flag, s);
    if (e != hipSuccess) return hip_fail(e, "check_nbr launch");
    int host_flag = 0;
    e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "check_nbr copy");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "check_nbr sync");
    if (host_flag) return fail(SSE_ERR_NBR, "neighbour table has an entry outside [0, %lld)", (long long)d.na);
    return ok();
}

}  // extern "C"
