// LDS-resident mixed-radix (2, 3, 4, 8) Stockham FFT over C interleaved lines.
//
// Element i of line c lives at s[i*C + c].  Each stage reads the RAD inputs of
// its butterflies into registers, synchronises, and writes the outputs in the
// Stockham order, so the result is in natural order without a bit reversal.
// Twiddles come from a table of W_N^m = exp(-2 pi i m / N), m < N, read with a
// compile-time stride TWS so that one table serves lengths N and N/2.
#pragma once
#include "common.h"

namespace ibdl {

constexpr int radix_for(int rem) {
    int a = 0, b = 0, t = rem;
    while (t % 2 == 0) { t /= 2; ++a; }
    while (t % 3 == 0) { t /= 3; ++b; }
    if (b > 0) return 3;
    if (a % 3 == 0) return 8;
    if (a == 1) return 2;
    return 4;
}

constexpr bool fft_size_ok(int n) {
    if (n < 2) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// Length-RAD DFT in registers; SIGN = -1 forward, +1 inverse (unnormalised).
template <int RAD, int SIGN, typename R>
__device__ __forceinline__ void butterfly(cplx<R>* v) {
    if constexpr (RAD == 2) {
        cplx<R> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (RAD == 3) {
        const R c1 = R(-0.5);
        const R s1 = R(0.86602540378443864676);  // sqrt(3)/2
        cplx<R> t = cadd(v[1], v[2]);
        cplx<R> d = csub(v[1], v[2]);
        cplx<R> m = {v[0].x + c1 * t.x, v[0].y + c1 * t.y};
        cplx<R> id = cmul_si<SIGN>(cscale(d, s1));
        v[0] = cadd(v[0], t);
        v[1] = cadd(m, id);
        v[2] = csub(m, id);
    } else if constexpr (RAD == 4) {
        cplx<R> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        cplx<R> t2 = cadd(v[1], v[3]), t3 = cmul_si<SIGN>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    } else {  // RAD == 8: two length-4 DFTs of the even and odd samples
        static_assert(RAD == 8, "radix");
        cplx<R> e[4] = {v[0], v[2], v[4], v[6]};
        cplx<R> o[4] = {v[1], v[3], v[5], v[7]};
        butterfly<4, SIGN>(e);
        butterfly<4, SIGN>(o);
        const R h = R(0.70710678118654752440);
        // W8^k = exp(SIGN * 2 pi i k / 8)
        cplx<R> w1 = cmul(o[1], cplx<R>{h, SIGN * h});
        cplx<R> w2 = cmul_si<SIGN>(o[2]);
        cplx<R> w3 = cmul(o[3], cplx<R>{-h, SIGN * h});
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], w1);
        v[5] = csub(e[1], w1);
        v[2] = cadd(e[2], w2);
        v[6] = csub(e[2], w2);
        v[3] = cadd(e[3], w3);
        v[7] = csub(e[3], w3);
    }
}

template <typename R, int L, int C, int T, int RAD, int NS, int SIGN, int TWS>
__device__ __forceinline__ void fft_stage(cplx<R>* s, const cplx<R>* __restrict__ tw) {
    constexpr int NB = L / RAD;     // butterflies per line
    constexpr int TOT = NB * C;     // butterflies in the block
    constexpr int PER = (TOT + T - 1) / T;
    cplx<R> v[PER][RAD];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int id = threadIdx.x + b * T;
        if (TOT % T == 0 || id < TOT) {
            const int c = id % C, j = id / C;
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[b][r] = s[(j + r * NB) * C + c];
            if constexpr (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < RAD; ++r) {
                    cplx<R> w = tw[(L / (NS * RAD)) * r * k * TWS];
                    if (SIGN > 0) w.y = -w.y;
                    v[b][r] = cmul(v[b][r], w);
                }
            }
            butterfly<RAD, SIGN>(v[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int id = threadIdx.x + b * T;
        if (TOT % T == 0 || id < TOT) {
            const int c = id % C, j = id / C;
            const int base = (j / NS) * NS * RAD + (j % NS);
#pragma unroll
            for (int r = 0; r < RAD; ++r) s[(base + r * NS) * C + c] = v[b][r];
        }
    }
    __syncthreads();
}

// Full length-L transform of the C lines held in s (natural order in and out).
template <typename R, int L, int C, int T, int SIGN, int TWS, int NS = 1, int REM = L>
__device__ __forceinline__ void fft_lines(cplx<R>* s, const cplx<R>* __restrict__ tw) {
    if constexpr (REM > 1) {
        constexpr int RAD = radix_for(REM);
        fft_stage<R, L, C, T, RAD, NS, SIGN, TWS>(s, tw);
        fft_lines<R, L, C, T, SIGN, TWS, NS * RAD, REM / RAD>(s, tw);
    }
}

}  // namespace ibdl
