// Shared device/host helpers of libsse (HIP, gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sse.h"

namespace sse {

// complex128 held as a pair of doubles (memory layout of interleaved re, im)
struct cd {
    double re, im;
};

__device__ __forceinline__ cd cload(const double* p, int64_t idx) {
    const double2 v = *reinterpret_cast<const double2*>(p + 2 * idx);
    return cd{v.x, v.y};
}
__device__ __forceinline__ void cstore(double* p, int64_t idx, cd v) {
    *reinterpret_cast<double2*>(p + 2 * idx) = make_double2(v.re, v.im);
}
__device__ __forceinline__ cd cmul(cd a, cd b) {
    return cd{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// acc += a * b
__device__ __forceinline__ void cfma(cd& acc, cd a, cd b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// acc += a * conj(b)
__device__ __forceinline__ void cfma_conj(cd& acc, cd a, cd b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.im, b.re, acc.im);
    acc.im = fma(-a.re, b.im, acc.im);
}
// acc += conj(a) * b
__device__ __forceinline__ void cfma_conja(cd& acc, cd a, cd b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}

// Plain-struct copy of the dims, passed by value to kernels.
struct Dims {
    int64_t nkz, ne, nqz, nw, na, nb, norb, gs;
};

inline Dims to_dims(const sse_dims& d) {
    return Dims{d.nkz, d.ne, d.nqz, d.nw, d.na, d.nb, d.norb, d.g_slots};
}

// Flat element offsets (in complex elements) of the tensors of the ABI.
__host__ __device__ __forceinline__ int64_t off_G(const Dims& d, int64_t k, int64_t e, int64_t b) {
    return (((k * d.ne + e) * d.na + b) * d.gs) * d.norb * d.norb;
}
__host__ __device__ __forceinline__ int64_t off_D(const Dims& d, int64_t q, int64_t w, int64_t a, int64_t n) {
    return (((q * d.nw + w) * d.na + a) * d.nb + n) * 9;
}
__host__ __device__ __forceinline__ int64_t off_A(const Dims& d, int64_t a, int64_t n, int i) {
    return ((a * d.nb + n) * 3 + i) * d.norb * d.norb;
}
__host__ __device__ __forceinline__ int64_t off_S(const Dims& d, int64_t k, int64_t e, int64_t a) {
    return ((k * d.ne + e) * d.na + a) * d.norb * d.norb;
}

}  // namespace sse
