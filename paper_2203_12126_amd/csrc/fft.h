// Mixed-radix Stockham FFT over C interleaved lines, register-resident stages.
//
// A length-L transform is split into S stages of radix R_1..R_S (each a product
// of 2s and 3s, at most RMAX).  In a stage every thread owns whole butterflies:
// it loads the RAD inputs of a butterfly into registers, multiplies by the
// stage twiddles, runs a length-RAD DFT in registers (itself split into radix
// 2/3/4/8 pieces with internal twiddles) and stores the outputs in Stockham
// order, so the result is in natural order without a bit reversal.  Stages pass
// data through LDS; the first stage may read straight from global memory and
// the last may write straight to global memory through the load/store functors.
//
// Element i of line c is addressed as (i, c); LDS holds it at s[i*C + c].
// Twiddles come from one table W_NT^m = exp(-2 pi i m / NT), m < NT, where NT
// is a multiple of every length used with it.
#pragma once
#include <utility>

#include "common.h"

namespace ibdl {

// ------------------------------------------------------------------ radix plans
constexpr bool smooth23(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

constexpr bool splittable(int L, int S, int RMAX) {
    if (S == 1) return L >= 2 && L <= RMAX && smooth23(L);
    for (int d = 2; d <= RMAX; ++d)
        if (L % d == 0 && smooth23(d) && splittable(L / d, S - 1, RMAX)) return true;
    return false;
}

struct RadixPlan {
    int n = 0;
    int r[4] = {1, 1, 1, 1};
};

constexpr double cpow(double x, int e) {
    double v = 1.0;
    for (int i = 0; i < e; ++i) v *= x;
    return v;
}

// fewest stages, then factors as close as possible to the geometric mean
constexpr RadixPlan make_plan(int L, int RMAX) {
    RadixPlan p{};
    int S = 1;
    while (S < 4 && !splittable(L, S, RMAX)) ++S;
    int rem = L;
    for (int s = 0; s < S; ++s) {
        const int left = S - s;
        if (left == 1) {
            p.r[s] = rem;
            break;
        }
        int best = -1;
        double bestq = 1e300;
        for (int d = 2; d <= RMAX; ++d) {
            if (rem % d || !smooth23(d) || !splittable(rem / d, left - 1, RMAX)) continue;
            const double a = cpow((double)d, left), b = (double)rem;
            const double q = a > b ? a / b : b / a;
            if (q < bestq) { bestq = q; best = d; }
        }
        p.r[s] = best;
        rem /= best;
    }
    p.n = S;
    return p;
}

constexpr int plan_max(const RadixPlan& p) {
    int m = 1;
    for (int i = 0; i < p.n; ++i) m = p.r[i] > m ? p.r[i] : m;
    return m;
}

template <int... Rs>
struct Radices {};

template <int L, int RMAX, size_t... I>
constexpr auto radices_fwd(std::index_sequence<I...>) -> Radices<make_plan(L, RMAX).r[I]...> {
    return {};
}
template <int L, int RMAX, size_t... I>
constexpr auto radices_rev(std::index_sequence<I...>)
    -> Radices<make_plan(L, RMAX).r[make_plan(L, RMAX).n - 1 - I]...> {
    return {};
}
template <int L, int RMAX>
using FwdRadices = decltype(radices_fwd<L, RMAX>(std::make_index_sequence<make_plan(L, RMAX).n>{}));
template <int L, int RMAX>
using RevRadices = decltype(radices_rev<L, RMAX>(std::make_index_sequence<make_plan(L, RMAX).n>{}));

// ------------------------------------------------------------------ register DFTs
// Length-RAD DFT of the base radices; SIGN = -1 forward, +1 inverse (unnormalised).
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
        cplx<R> m = {fmac(c1, t.x, v[0].x), fmac(c1, t.y, v[0].y)};
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
    } else {
        static_assert(RAD == 8, "radix");
        cplx<R> e[4] = {v[0], v[2], v[4], v[6]};
        cplx<R> o[4] = {v[1], v[3], v[5], v[7]};
        butterfly<4, SIGN>(e);
        butterfly<4, SIGN>(o);
        const R h = R(0.70710678118654752440);
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

// exp(-2 pi i m / n) at compile time: the angle is reduced exactly in integers to
// phi in [0, pi/4] (quarter turns and the complement), then sin/cos of phi by
// their Taylor series.
struct CD {
    double re, im;
};
constexpr CD expm2pi(long m, long n) {
    m %= n;
    if (m < 0) m += n;
    const long q = (4 * m) / n;          // quarter turns
    const long r = 4 * m - q * n;        // remaining angle (pi/2) r/n
    const bool comp = 2 * r > n;
    const long rr = comp ? n - r : r;
    const double phi = 1.57079632679489661923132169163975144 * (double)rr / (double)n;
    double s = 0.0, c = 0.0, ts = phi, tc = 1.0;
    for (int k = 1; k < 15; ++k) {
        s += ts;
        ts *= -phi * phi / (double)((2 * k) * (2 * k + 1));
        c += tc;
        tc *= -phi * phi / (double)((2 * k - 1) * (2 * k));
    }
    if (comp) {
        const double t = s;
        s = c;
        c = t;
    }
    for (long i = 0; i < q; ++i) {
        const double t = c;
        c = -s;
        s = t;
    }
    return CD{c, -s};
}
template <int RAD>
struct TwTab {
    double re[RAD > 0 ? RAD : 1];
    double im[RAD > 0 ? RAD : 1];
};
template <int RAD>
constexpr TwTab<RAD> make_twtab() {
    TwTab<RAD> t{};
    for (int m = 0; m < RAD; ++m) {
        const CD w = expm2pi(m, RAD);
        t.re[m] = w.re;
        t.im[m] = w.im;
    }
    return t;
}
template <int RAD>
struct TwConst {
    static constexpr TwTab<RAD> tab = make_twtab<RAD>();
};

__device__ __forceinline__ int imin_c(int a, int b) { return a < b ? a : b; }

// Stage twiddles W^idx (W = exp(-2 pi i / NT)) from two small LDS tables:
// lo[i] = W^i for i < 64 and hi[j] = W^(64 j), W^idx = lo[idx % 64] hi[idx / 64].
template <typename R>
struct Tw2 {
    const cplx<R>* lo;
    const cplx<R>* hi;
    __device__ __forceinline__ cplx<R> get(int idx) const { return cmul(lo[idx & 63], hi[idx >> 6]); }
};
template <int NT>
struct Tw2Size {
    static constexpr int LO = NT < 64 ? NT : 64;
    static constexpr int HI = (NT + 63) / 64;
    static constexpr int ALL = LO + HI;
};
// fills the tables from the full table tw[0..NT) (call before a barrier)
template <typename R, int NT, int T>
__device__ __forceinline__ Tw2<R> load_tw2(cplx<R>* lds, const cplx<R>* __restrict__ tw) {
    using S = Tw2Size<NT>;
    // every element loaded (clamped index), so the array stays in registers
    cplx<R> v[(S::ALL + T - 1) / T];
#pragma unroll
    for (int u = 0; u < (S::ALL + T - 1) / T; ++u) {
        const int i = imin_c(threadIdx.x + u * T, S::ALL - 1);
        v[u] = tw[i < S::LO ? i : 64 * (i - S::LO)];
    }
#pragma unroll
    for (int u = 0; u < (S::ALL + T - 1) / T; ++u) {
        const int i = threadIdx.x + u * T;
        if (i < S::ALL) lds[i] = v[u];
    }
    return Tw2<R>{lds, lds + S::LO};
}

// The full table W^idx, idx < NT, in LDS (when it fits the kernel's LDS budget).
template <typename R>
struct TwFull {
    const cplx<R>* tab;
    __device__ __forceinline__ cplx<R> get(int idx) const { return tab[idx]; }
};
template <typename R, int NT, int T>
__device__ __forceinline__ TwFull<R> load_twfull(cplx<R>* lds, const cplx<R>* __restrict__ tw) {
    constexpr int P = (NT + T - 1) / T;
    cplx<R> v[P];  // every element loaded (clamped index), so the array stays in registers
#pragma unroll
    for (int u = 0; u < P; ++u) v[u] = tw[imin_c(threadIdx.x + u * T, NT - 1)];
#pragma unroll
    for (int u = 0; u < P; ++u) {
        const int i = threadIdx.x + u * T;
        if (i < NT) lds[i] = v[u];
    }
    return TwFull<R>{lds};
}
// LDS twiddle storage: the full table or the two small ones
template <typename R, int NT, bool FULL>
struct TwLds;
template <typename R, int NT>
struct TwLds<R, NT, true> {
    using type = TwFull<R>;
    static constexpr int SIZE = NT;
    template <int T>
    __device__ __forceinline__ static type load(cplx<R>* lds, const cplx<R>* tw) { return load_twfull<R, NT, T>(lds, tw); }
};
template <typename R, int NT>
struct TwLds<R, NT, false> {
    using type = Tw2<R>;
    static constexpr int SIZE = Tw2Size<NT>::ALL;
    template <int T>
    __device__ __forceinline__ static type load(cplx<R>* lds, const cplx<R>* tw) { return load_tw2<R, NT, T>(lds, tw); }
};

template <int SIGN, class TW>
__device__ __forceinline__ auto twiddle(const TW& tw, int idx) {
    auto w = tw.get(idx);
    if (SIGN > 0) w.y = -w.y;
    return w;
}

// Length-RAD DFT in registers.  RAD = R1 * R2 with R1 a base radix:
//   X[k1 + R1 k2] = sum_n2 W_RAD^{n2 k1} W_R2^{n2 k2} sum_n1 x[R2 n1 + n2] W_R1^{n1 k1}.
template <int RAD, int SIGN, typename R>
__device__ __forceinline__ void reg_dft(cplx<R>* v) {
    if constexpr (RAD == 2 || RAD == 3 || RAD == 4 || RAD == 8) {
        butterfly<RAD, SIGN>(v);
    } else {
        constexpr int R1 = (RAD % 8 == 0) ? 8 : (RAD % 4 == 0) ? 4 : (RAD % 2 == 0) ? 2 : 3;
        constexpr int R2 = RAD / R1;
        cplx<R> a[R2][R1];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) a[n2][n1] = v[R2 * n1 + n2];
            butterfly<R1, SIGN>(a[n2]);
        }
#pragma unroll
        for (int n2 = 1; n2 < R2; ++n2)
#pragma unroll
            for (int k1 = 1; k1 < R1; ++k1) {
                const int e = n2 * k1;
                const cplx<R> w = {(R)TwConst<RAD>::tab.re[e], (R)(-SIGN * TwConst<RAD>::tab.im[e])};
                a[n2][k1] = cmul(a[n2][k1], w);
            }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            cplx<R> b[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) b[n2] = a[n2][k1];
            reg_dft<R2, SIGN>(b);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = b[k2];
        }
    }
}

// ------------------------------------------------------------------ stages
// LDS layouts of a transform's rows: idx(i, c) is the element index of column c
// (one of C) of row i.
//
// PadRows: row-major with one padding row after every 2^PS rows (PS = 0: none).
// The first stage of a transform writes rows RAD apart; with RAD = 2^PS the
// padding moves consecutive butterflies' rows to different LDS banks.
template <int C, int PS = 0>
struct PadRows {
    static constexpr int rows(int L) { return PS == 0 ? L : L + ((L - 1) >> PS) + 1; }
    __device__ __forceinline__ static constexpr int idx(int i, int c) {
        if constexpr (PS == 0) return i * C + c;
        else return (i + (i >> PS)) * C + c;
    }
};
// XorRows: row-major and unpadded, column c of row i held at column c ^ g(i), where
// g(i) is the XOR of M_b over the set bits b of i (every M_b < C, so a row keeps
// its C slots).  Rows that one instruction touches in the same column then sit in
// different banks.
template <int C, int M0, int M1, int M2, int M3, int M4>
struct XorRows {
    static constexpr int rows(int L) { return L; }
    __device__ __forceinline__ static constexpr int g(int i) {
        return ((i & 1) ? M0 : 0) ^ ((i & 2) ? M1 : 0) ^ ((i & 4) ? M2 : 0) ^ ((i & 8) ? M3 : 0) ^
               ((i & 16) ? M4 : 0);
    }
    __device__ __forceinline__ static constexpr int idx(int i, int c) { return i * C + (c ^ g(i)); }
};

// LDS functors over a layout
template <typename R, class LAY>
struct LdsLoad {
    const cplx<R>* s;
    __device__ __forceinline__ cplx<R> operator()(int i, int c) const { return s[LAY::idx(i, c)]; }
};
template <typename R, class LAY>
struct LdsStore {
    cplx<R>* s;
    __device__ __forceinline__ void operator()(int i, int c, cplx<R> v) const { s[LAY::idx(i, c)] = v; }
};

constexpr bool is_pow2(int a) { return a > 0 && (a & (a - 1)) == 0; }

// Every stage hands output slot k = b * RAD + r of a thread (its b-th butterfly,
// r-th output) to the store functor through store_out; a functor that needs the
// slot (values prefetched per output) overloads it.
template <class ST, typename R>
__device__ __forceinline__ void store_out(ST& st, int i, int c, cplx<R> v, int) {
    st(i, c, v);
}

// The last radix of a plan: its stage writes row j + r * (L / RAD) of column c for
// the butterfly id = j * C + c (NS * RAD = L there).
template <int L, int RMAX>
constexpr int last_radix() {
    return make_plan(L, RMAX).r[make_plan(L, RMAX).n - 1];
}

// One stage: TH threads cover the C*L/RAD butterflies, PER per thread.  A thread's
// rows are j + r NB (loads, j < NB) and base + r NS (stores, base % NS < NS and
// base a multiple of NS RAD above that); with power-of-two sizes the two terms
// share no bits and the sum is written as an OR, so that a layout's function of
// the row bits splits into a per-butterfly part and a per-r constant.
template <typename R, int L, int C, int TH, int NT, int SIGN, class LAY, int NS, int RAD, int... REST, class TW,
          class LD, class ST>
__device__ __forceinline__ void run_stages(cplx<R>* s, const TW& tw, LD ld, ST st) {
    constexpr int NB = L / RAD;
    constexpr int TOT = NB * C;
    constexpr int PER = (TOT + TH - 1) / TH;
    cplx<R> v[PER][RAD];
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int id = threadIdx.x + b * TH;
        if (TOT % TH == 0 || id < TOT) {
            const int c = id % C, j = id / C;
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[b][r] = ld(is_pow2(NB) ? (j | (r * NB)) : (j + r * NB), c);
            if constexpr (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < RAD; ++r)
                    v[b][r] = cmul(v[b][r], twiddle<SIGN>(tw, (NT / (NS * RAD)) * r * k));
            }
            reg_dft<RAD, SIGN>(v[b]);
        }
    }
    auto emit = [&](auto&& out) {
#pragma unroll
        for (int b = 0; b < PER; ++b) {
            const int id = threadIdx.x + b * TH;
            if (TOT % TH == 0 || id < TOT) {
                const int c = id % C, j = id / C;
                const int base = (j / NS) * NS * RAD + (j % NS);
#pragma unroll
                for (int r = 0; r < RAD; ++r)
                    store_out(out, is_pow2(NS) && is_pow2(RAD) ? (base | (r * NS)) : (base + r * NS), c, v[b][r],
                              b * RAD + r);
            }
        }
    };
    if constexpr (sizeof...(REST) == 0) {
        __syncthreads();  // the store may overwrite LDS this stage (or a caller) read
        emit(st);
    } else {
        __syncthreads();  // every input of this stage has been read
        emit(LdsStore<R, LAY>{s});
        __syncthreads();
        run_stages<R, L, C, TH, NT, SIGN, LAY, NS * RAD, REST...>(s, tw, LdsLoad<R, LAY>{s}, st);
    }
}

// LAY: layout of the intermediate LDS rows; the caller's functors use the same
// layout where they touch those rows.
template <typename R, int L, int C, int TH, int NT, int SIGN, class LAY = PadRows<C>, class TW, class LD, class ST,
          int... Rs>
__device__ __forceinline__ void run_fft(cplx<R>* s, const TW& tw, LD ld, ST st, Radices<Rs...>) {
    run_stages<R, L, C, TH, NT, SIGN, LAY, 1, Rs...>(s, tw, ld, st);
}

// log2 of the first radix of a plan when it is a power of two >= 4, else 0
template <int L, int RMAX>
constexpr int first_radix_shift() {
    const int r = make_plan(L, RMAX).r[0];
    int sh = 0;
    while ((1 << sh) < r) ++sh;
    return ((1 << sh) == r && r >= 4 && make_plan(L, RMAX).n > 1) ? sh : 0;
}

// Threads per block so that the largest radix stage has one butterfly per thread.
template <int L, int C, int RMAX>
constexpr int fft_threads() {
    constexpr int t = C * L / plan_max(make_plan(L, RMAX));
    return t < 64 ? 64 : (t > 1024 ? 1024 : (t + 63) / 64 * 64);
}

}  // namespace ibdl
