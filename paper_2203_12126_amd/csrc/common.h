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

// The library is built without floating-point contraction (-ffp-contract=off), so
// every multiply-add that should be fused says so (fmac): the rounding of each
// result then does not depend on how the compiler schedules a kernel's code, and
// every workgroup shape of a pass gives bit-identical results.
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {fmac(a.x, b.x, -(a.y * b.y)), fmac(a.x, b.y, a.y * b.x)};
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

// Raw buffer access within one range [base, base + bytes) given by a buffer
// descriptor: a 32-bit byte offset per lane; an offset at or beyond `bytes`
// reads as zero and drops the store (the buffer unit's range check), so masked
// elements need no branch.  bytes < 2^31.
constexpr int kBufOut = 0x7ffffff0;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
    // word 3: 32-bit data format, as untyped buffer loads and stores require on gfx9
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// one real through a buffer descriptor (offset in bytes; past the range: 0)
template <typename R>
struct BufScalar;
template <>
struct BufScalar<float> {
    __device__ __forceinline__ static float load(__amdgpu_buffer_rsrc_t r, int off) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
};
template <>
struct BufScalar<double> {
    typedef unsigned int V __attribute__((ext_vector_type(2)));
    __device__ __forceinline__ static double load(__amdgpu_buffer_rsrc_t r, int off) {
        const V v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return __longlong_as_double((long long)(((unsigned long long)v.y << 32) | v.x));
    }
};
template <typename R>
struct BufIO;
template <>
struct BufIO<float> {
    typedef unsigned int V __attribute__((ext_vector_type(2)));
    __device__ __forceinline__ static cplx<float> load(__amdgpu_buffer_rsrc_t r, int off) {
        const V v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return {__uint_as_float(v.x), __uint_as_float(v.y)};
    }
    __device__ __forceinline__ static void store(__amdgpu_buffer_rsrc_t r, int off, cplx<float> c) {
        const V v = {__float_as_uint(c.x), __float_as_uint(c.y)};
        __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
    }
};
template <>
struct BufIO<double> {
    typedef unsigned int V __attribute__((ext_vector_type(4)));
    __device__ __forceinline__ static cplx<double> load(__amdgpu_buffer_rsrc_t r, int off) {
        const V v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const unsigned long long a = ((unsigned long long)v.y << 32) | v.x;
        const unsigned long long b = ((unsigned long long)v.w << 32) | v.z;
        return {__longlong_as_double((long long)a), __longlong_as_double((long long)b)};
    }
    __device__ __forceinline__ static void store(__amdgpu_buffer_rsrc_t r, int off, cplx<double> c) {
        const unsigned long long a = (unsigned long long)__double_as_longlong(c.x);
        const unsigned long long b = (unsigned long long)__double_as_longlong(c.y);
        const V v = {(unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32)};
        __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, 0);
    }
};

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
