// Shared device/host helpers of the IBDL HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace ibdl {

template <typename R>
struct __align__(2 * sizeof(R)) cplx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by s*i (s = +1 or -1)
template <int S, typename R>
__device__ __forceinline__ cplx<R> cmul_si(cplx<R> a) {
    return S > 0 ? cplx<R>{-a.y, a.x} : cplx<R>{a.y, -a.x};
}

// Discrete delta kernels (Sec. 5.2).  Peskin's four-point function:
//   phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8        0 <= |r| <= 1
//          = (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8       1 <= |r| <= 2
//          = 0                                               |r| >= 2
// and the cosine kernel phi(r) = (1 + cos(pi r / 2)) / 4 for |r| < 2.
__device__ __forceinline__ double phi_peskin4(double r) {
    double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
    if (a < 2.0) return (5.0 - 2.0 * a - sqrt(fmax(0.0, -7.0 + 12.0 * a - 4.0 * a * a))) * 0.125;
    return 0.0;
}
__device__ __forceinline__ double phi_cosine4(double r) {
    double a = fabs(r);
    return a < 2.0 ? 0.25 * (1.0 + cospi(0.5 * a)) : 0.0;
}

// Status plumbing (host side).
struct Error {
    int status;
    std::string msg;
};

}  // namespace ibdl

#define IBDL_HIP_TRY(expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::ibdl::Error{3, std::string(#expr) + ": " + hipGetErrorString(e_)};  \
    } while (0)
