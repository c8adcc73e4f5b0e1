// One pass of L^-1 through the periodic grid, fused with the spread on the way
// in and the interpolation on the way out (Sec. 5.2-5.3):
//
//   row_fwd : per x-line, build the line of the forcing in LDS (dense grid input
//             and/or the dipole/monopole spread from the sparse spread matrix,
//             each node summed in a fixed order), real-to-complex FFT along x
//             (length-n/2 complex FFT plus the split step), store the half
//             spectrum row;
//   col     : per group of C adjacent half-spectrum columns, FFT along y (2-D)
//             or y/z (3-D); the last axis multiplies by the inverse symbol of
//             L = Lap_h - alpha between its forward and inverse transforms;
//   row_inv : per x-line, complex-to-real inverse FFT along x, then either the
//             line of the grid solution is stored or every boundary point whose
//             4^d stencil touches the line adds its partial interpolation sum;
//   finish  : per boundary point, the fixed-order sum of its partials, scaled
//             and combined with an FP64 term (the +-q/2 of the operator).
//
// Lines without spread contributions are never written nor read (their
// spectrum rows are zero), and lines no boundary point interpolates from are
// not transformed back.
#pragma once
#include "fft.h"
#include "plan.h"

namespace ibdl {

constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int rup64(int x) { return (x + 63) / 64 * 64; }

// Column-group width: C adjacent complex columns are read per row (64 bytes).
template <typename R>
struct ColBytes { static constexpr int value = 64; };

template <typename R, int N>
struct RowCfg {
    static constexpr int L = N / 2;                            // complex length
    static constexpr int G = imax(1, imin(64, 2048 / L));       // lines per block
    static constexpr int T = imax(64, imin(1024, rup64(G * L / 8)));
};
template <typename R, int N>
struct ColCfg {
    static constexpr int C = ColBytes<R>::value / (2 * (int)sizeof(R));
    static constexpr int T = imax(64, imin(1024, rup64(N * C / 8)));
};

// ------------------------------------------------------------ accumulation
template <typename R>
struct Acc;
template <>
struct Acc<double> {
    double s = 0.0;
    __device__ __forceinline__ void add(double w, double q) { s = fma(w, q, s); }
    __device__ __forceinline__ double value() const { return s; }
};
// FP32 dot product with error-free transformations (TwoProduct by fma, TwoSum):
// the rounding errors of every product and partial sum are collected in c.
template <>
struct Acc<float> {
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float w, float q) {
#pragma clang fp contract(off)
        float p = w * q;
        float pe = fmaf(w, q, -p);
        float t = s + p;
        float bp = t - s;
        float se = (s - (t - bp)) + (p - bp);
        s = t;
        c = c + (se + pe);
    }
    __device__ __forceinline__ float value() const { return s + c; }
};

// ------------------------------------------------------------ arguments
template <typename R>
struct CsrView {
    const int32_t* line_act;
    const int32_t* act_ptr;
    const uint32_t* act_node;
    const uint32_t* k;
    const R* w;
    const double* q;     // q + rhs * q_stride: strengths of one right-hand side
    size_t q_stride;
    double coef;
};

template <typename R>
struct RowFwdArgs {
    const int32_t* lines;  // line list or null (identity)
    int nproc;
    int M;
    CsrView<R> dip, mono;
    const double* grid;    // [nrhs][n^dim] or null
    double cg;
    size_t grid_stride;
    cplx<R>* spec;
    size_t spec_stride;
    int P;
    const cplx<R>* tw;
};

template <typename R>
struct ColArgs {
    cplx<R>* spec;
    size_t rhs_stride;
    const int32_t* outer_list;
    size_t outer_stride;
    size_t elem_stride;
    int width;
    const uint8_t* lmask;
    int lm_outer, lm_stride;
    const uint8_t* smask;
    int sm_outer, sm_stride;
    const cplx<R>* tw;
    const R* s2;
    R alpha;
    R norm;
    int dim3;
};

template <typename R>
struct RowInvArgs {
    const int32_t* lines;
    int nproc;
    const cplx<R>* spec;
    size_t spec_stride;
    int P;
    const cplx<R>* tw;
    double* u;             // grid output [nrhs][n^dim]
    size_t u_stride;
    const int32_t* line_start;
    const int32_t* cell;   // [M][3] sorted order
    const R* taps;         // [M][3][4] sorted order
    R* part;               // [nrhs][M][gpp]
    size_t part_stride;
    int M;
    int dim;
};

// ------------------------------------------------------------ spread phase
// Adds coef * (sum_e w_e q[k_e]) into the LDS lines for every active node of
// the block's lines.  Each node is written by exactly one thread.
template <typename R, int N, int G, int T>
__device__ __forceinline__ void spread_phase(R* sr, const CsrView<R>& c, int rhs, int M,
                                             const int32_t* lines, int first, int nproc,
                                             int* rs) {
    if (threadIdx.x < G) {
        const int g = threadIdx.x;
        int cnt = 0;
        const int li = first + g;
        if (li < nproc) {
            const int line = lines ? lines[li] : li;
            cnt = c.line_act[line + 1] - c.line_act[line];
        }
        rs[g + 1] = cnt;
    }
    if (threadIdx.x == 0) rs[0] = 0;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int g = 1; g <= G; ++g) rs[g] += rs[g - 1];
    __syncthreads();
    const int total = rs[G];
    const double* q = c.q + (size_t)rhs * c.q_stride;
    for (int f = threadIdx.x; f < total; f += T) {
        int lo = 0, hi = G;  // find g with rs[g] <= f < rs[g+1]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (rs[mid] <= f) lo = mid; else hi = mid;
        }
        const int g = lo;
        const int line = lines ? lines[first + g] : first + g;
        const int a = c.line_act[line] + (f - rs[g]);
        const int x = (int)(c.act_node[a] - (uint32_t)line * (uint32_t)N);
        Acc<R> acc;
        const int e1 = c.act_ptr[a + 1];
        for (int e = c.act_ptr[a]; e < e1; ++e) acc.add(c.w[e], (R)q[c.k[e]]);
        sr[2 * ((x >> 1) * G + g) + (x & 1)] += (R)c.coef * acc.value();
    }
    __syncthreads();
}

// ------------------------------------------------------------ row_fwd
template <typename R, int N>
__global__ __launch_bounds__((RowCfg<R, N>::T)) void k_row_fwd(RowFwdArgs<R> a) {
    using CF = RowCfg<R, N>;
    constexpr int L = CF::L, G = CF::G, T = CF::T;
    __shared__ cplx<R> s[L * G];
    __shared__ int rs[G + 1];
    R* sr = reinterpret_cast<R*>(s);
    const int rhs = blockIdx.y;
    const int first = blockIdx.x * G;
    for (int i = threadIdx.x; i < L * G; i += T) s[i] = cplx<R>{R(0), R(0)};
    __syncthreads();
    if (a.grid) {
        const double* gr = a.grid + (size_t)rhs * a.grid_stride;
        for (int id = threadIdx.x; id < N * G; id += T) {
            const int g = id / N, x = id % N;
            const int li = first + g;
            if (li < a.nproc) {
                const int line = a.lines ? a.lines[li] : li;
                sr[2 * ((x >> 1) * G + g) + (x & 1)] = (R)(a.cg * gr[(size_t)line * N + x]);
            }
        }
        __syncthreads();
    }
    if (a.dip.q) spread_phase<R, N, G, T>(sr, a.dip, rhs, a.M, a.lines, first, a.nproc, rs);
    if (a.mono.q) spread_phase<R, N, G, T>(sr, a.mono, rhs, a.M, a.lines, first, a.nproc, rs);

    fft_lines<R, L, G, T, -1, 2>(s, a.tw);

    // split step: X[k] = (Z_k + conj Z_{L-k})/2 - i W_N^k (Z_k - conj Z_{L-k})/2
    cplx<R>* out = a.spec + (size_t)rhs * a.spec_stride;
    constexpr int H = L / 2 + 1;
    for (int id = threadIdx.x; id < G * H; id += T) {
        const int g = id / H, k = id % H;
        const int li = first + g;
        if (li >= a.nproc) continue;
        const int line = a.lines ? a.lines[li] : li;
        const cplx<R> zk = s[k * G + g];
        const cplx<R> zm = s[((L - k) % L) * G + g];
        const cplx<R> e = cscale(cadd(zk, cconj(zm)), R(0.5));
        const cplx<R> d = cscale(csub(zk, cconj(zm)), R(0.5));
        const cplx<R> o = cmul_si<-1>(d);                           // -i d
        const cplx<R> xk = cadd(e, cmul(a.tw[k], o));
        const cplx<R> xm = cadd(cconj(e), cmul(a.tw[L - k], cmul_si<-1>(cscale(cconj(d), R(-1)))));
        cplx<R>* row = out + (size_t)line * a.P;
        row[k] = xk;
        if (k != L - k) row[L - k] = xm;
    }
}

// ------------------------------------------------------------ col
// MODE 0: forward; 1: forward, times inverse symbol, inverse; 2: inverse.
template <typename R, int N, int MODE>
__global__ __launch_bounds__((ColCfg<R, N>::T)) void k_col(ColArgs<R> a) {
    constexpr int C = ColCfg<R, N>::C, T = ColCfg<R, N>::T;
    __shared__ cplx<R> s[N * C];
    const int grp = blockIdx.x;
    const int outer = a.outer_list ? a.outer_list[blockIdx.y] : (int)blockIdx.y;
    const int rhs = blockIdx.z;
    cplx<R>* base = a.spec + (size_t)rhs * a.rhs_stride + (size_t)outer * a.outer_stride + (size_t)grp * C;
    const int ncol = imin(C, a.width - grp * C);
    for (int id = threadIdx.x; id < N * C; id += T) {
        const int c = id % C, i = id / C;
        cplx<R> v = {R(0), R(0)};
        if (c < ncol && (!a.lmask || a.lmask[outer * a.lm_outer + i * a.lm_stride]))
            v = base[(size_t)i * a.elem_stride + c];
        s[i * C + c] = v;
    }
    __syncthreads();
    if constexpr (MODE == 2) {
        fft_lines<R, N, C, T, +1, 1>(s, a.tw);
    } else {
        fft_lines<R, N, C, T, -1, 1>(s, a.tw);
    }
    if constexpr (MODE == 1) {
        // multiply by norm / lambda(k), lambda = -(sum_d (4/h^2) sin^2(pi k_d/n)) - alpha
        for (int id = threadIdx.x; id < N * C; id += T) {
            const int c = id % C, i = id / C;
            if (c < ncol) {
                const int kx = grp * C + c;
                const R lam = a.s2[kx] + a.s2[i] + (a.dim3 ? a.s2[outer] : R(0)) + a.alpha;
                const R sig = lam != R(0) ? -a.norm / lam : R(0);
                s[i * C + c] = cscale(s[i * C + c], sig);
            }
        }
        __syncthreads();
        fft_lines<R, N, C, T, +1, 1>(s, a.tw);
    }
    for (int id = threadIdx.x; id < N * C; id += T) {
        const int c = id % C, i = id / C;
        if (c < ncol && (!a.smask || a.smask[outer * a.sm_outer + i * a.sm_stride]))
            base[(size_t)i * a.elem_stride + c] = s[i * C + c];
    }
}

// ------------------------------------------------------------ row_inv
// OUT 0: interpolation partial sums; OUT 1: grid output.
template <typename R, int N, int OUT>
__global__ __launch_bounds__((RowCfg<R, N>::T)) void k_row_inv(RowInvArgs<R> a) {
    using CF = RowCfg<R, N>;
    constexpr int L = CF::L, G = CF::G, T = CF::T;
    __shared__ cplx<R> s[L * G];
    R* sr = reinterpret_cast<R*>(s);
    const int rhs = blockIdx.y;
    const int first = blockIdx.x * G;
    const cplx<R>* spec = a.spec + (size_t)rhs * a.spec_stride;
    // inverse split step: Z_k = (X_k + conj X_{L-k})/2 + i W_N^-k (X_k - conj X_{L-k})/2
    for (int id = threadIdx.x; id < G * L; id += T) {
        const int g = id / L, k = id % L;
        const int li = first + g;
        cplx<R> z = {R(0), R(0)};
        if (li < a.nproc) {
            const int line = a.lines ? a.lines[li] : li;
            const cplx<R>* row = spec + (size_t)line * a.P;
            const cplx<R> xk = row[k];
            const cplx<R> xm = row[L - k];
            const cplx<R> e = cscale(cadd(xk, cconj(xm)), R(0.5));
            const cplx<R> d = cscale(csub(xk, cconj(xm)), R(0.5));
            z = cadd(e, cmul_si<1>(cmul(cconj(a.tw[k]), d)));
        }
        s[k * G + g] = z;
    }
    __syncthreads();
    fft_lines<R, L, G, T, +1, 2>(s, a.tw);

    if constexpr (OUT == 1) {
        double* u = a.u + (size_t)rhs * a.u_stride;
        for (int id = threadIdx.x; id < G * N; id += T) {
            const int g = id / N, x = id % N;
            const int li = first + g;
            if (li < a.nproc) {
                const int line = a.lines ? a.lines[li] : li;
                u[(size_t)line * N + x] = (double)sr[2 * ((x >> 1) * G + g) + (x & 1)];
            }
        }
    } else {
        R* part = a.part + (size_t)rhs * a.part_stride;
        const int gpp = a.dim == 3 ? 16 : 4;
        for (int g = 0; g < G; ++g) {
            const int li = first + g;
            if (li >= a.nproc) break;
            const int line = a.lines ? a.lines[li] : li;
            const int y = line % N, z = line / N;
            // sorted-point ranges of the x-lines (cy, cz) with cy in y-2..y+1, cz in z-2..z+1
            int rb[8], rc[8], nr = 0;
            const int nz = a.dim == 3 ? 4 : 1;
            for (int dz = 0; dz < nz; ++dz) {
                const int cz = a.dim == 3 ? (z - 2 + dz + N) % N : 0;
                const int pz = cz * N;
                const int lo = y - 2, hi = y + 2;
                if (lo < 0) {
                    rb[nr] = a.line_start[pz + lo + N];
                    rc[nr] = a.line_start[pz + N] - rb[nr]; ++nr;
                    rb[nr] = a.line_start[pz];
                    rc[nr] = a.line_start[pz + hi] - rb[nr]; ++nr;
                } else if (hi > N) {
                    rb[nr] = a.line_start[pz + lo];
                    rc[nr] = a.line_start[pz + N] - rb[nr]; ++nr;
                    rb[nr] = a.line_start[pz];
                    rc[nr] = a.line_start[pz + hi - N] - rb[nr]; ++nr;
                } else {
                    rb[nr] = a.line_start[pz + lo];
                    rc[nr] = a.line_start[pz + hi] - rb[nr]; ++nr;
                }
            }
            int total = 0;
            for (int r = 0; r < nr; ++r) total += rc[r];
            for (int f = threadIdx.x; f < total; f += T) {
                int r = 0, off = f;
                while (off >= rc[r]) { off -= rc[r]; ++r; }
                const int sidx = rb[r] + off;
                const int cx = a.cell[3 * sidx + 0];
                const int cy = a.cell[3 * sidx + 1];
                const int oy = (y - cy + 1 + N) % N;
                const R* tp = a.taps + (size_t)sidx * 12;
                R acc = R(0);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int x = (cx - 1 + t + N) % N;
                    acc += tp[t] * sr[2 * ((x >> 1) * G + g) + (x & 1)];
                }
                acc *= tp[4 + oy];
                int o = oy;
                if (a.dim == 3) {
                    const int cz = a.cell[3 * sidx + 2];
                    const int oz = (z - cz + 1 + N) % N;
                    acc *= tp[8 + oz];
                    o += 4 * oz;
                }
                part[(size_t)sidx * gpp + o] = acc;
            }
        }
    }
}

// ------------------------------------------------------------ finish
struct FinishArgs {
    const uint32_t* perm;
    int M, gpp;
    size_t part_stride;
    double* out;
    size_t out_stride;
    double cA;
    const double* in;
    size_t in_stride;
    double cB;
    const double* in2;
    size_t in2_stride;
    double cC;
};

template <typename R>
__global__ void k_finish(const R* __restrict__ part, FinishArgs f) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (s >= f.M) return;
    const R* p = part + (size_t)rhs * f.part_stride + (size_t)s * f.gpp;
    double acc = 0.0;
    for (int o = 0; o < f.gpp; ++o) acc += (double)p[o];
    const uint32_t k = f.perm[s];
    double v = f.cA * acc;
    if (f.in) v += f.cB * f.in[(size_t)rhs * f.in_stride + k];
    if (f.in2) v += f.cC * f.in2[(size_t)rhs * f.in2_stride + k];
    f.out[(size_t)rhs * f.out_stride + k] = v;
}

// ------------------------------------------------------------ dispatch
#define IBDL_SIZES(X) \
    X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048)

template <typename R>
inline int row_lines_per_block(int n) {
    switch (n) {
#define IBDL_C(NN) case NN: return RowCfg<R, NN>::G;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
    return 1;
}
template <typename R>
inline int col_width(int n) {
    switch (n) {
#define IBDL_C(NN) case NN: return ColCfg<R, NN>::C;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
    return 1;
}

template <typename R>
void launch_row_fwd(int n, dim3 grid, hipStream_t st, const RowFwdArgs<R>& a) {
    switch (n) {
#define IBDL_C(NN) \
    case NN: hipLaunchKernelGGL((k_row_fwd<R, NN>), grid, dim3(RowCfg<R, NN>::T), 0, st, a); break;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
}
template <typename R, int MODE>
void launch_col(int n, dim3 grid, hipStream_t st, const ColArgs<R>& a) {
    switch (n) {
#define IBDL_C(NN) \
    case NN: hipLaunchKernelGGL((k_col<R, NN, MODE>), grid, dim3(ColCfg<R, NN>::T), 0, st, a); break;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
}
template <typename R, int OUT>
void launch_row_inv(int n, dim3 grid, hipStream_t st, const RowInvArgs<R>& a) {
    switch (n) {
#define IBDL_C(NN) \
    case NN: hipLaunchKernelGGL((k_row_inv<R, NN, OUT>), grid, dim3(RowCfg<R, NN>::T), 0, st, a); break;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
}

template <typename R>
struct PlanPrec;
template <>
struct PlanPrec<double> {
    static const double* w(const Csr& c) { return c.w64; }
    static const double* taps(ibdl_plan p) { return p->taps64; }
    static const cplx<double>* tw(ibdl_plan p) { return reinterpret_cast<const cplx<double>*>(p->tw64); }
    static const double* s2(ibdl_plan p) { return p->s2_64; }
};
template <>
struct PlanPrec<float> {
    static const float* w(const Csr& c) { return c.w32; }
    static const float* taps(ibdl_plan p) { return p->taps32; }
    static const cplx<float>* tw(ibdl_plan p) { return reinterpret_cast<const cplx<float>*>(p->tw32); }
    static const float* s2(ibdl_plan p) { return p->s2_32; }
};

template <typename R>
void run_pipeline_t(ibdl_plan p, int nrhs, const PipeIn& in, const PipeOut& out, hipStream_t st) {
    using PP = PlanPrec<R>;
    const int n = p->n;
    const bool dense_in = in.grid != nullptr;
    const bool dense_out = out.u != nullptr;
    cplx<R>* spec = reinterpret_cast<cplx<R>*>(p->ws.spec);
    const size_t sstride = p->spec_elems;
    int stage = 0;

    // ---- row_fwd
    RowFwdArgs<R> ra{};
    ra.lines = dense_in ? nullptr : p->spread_lines;
    ra.nproc = dense_in ? p->nlines : p->n_spread_lines;
    ra.M = p->M;
    auto view = [&](const Csr& c, const double* q, double coef) {
        CsrView<R> v{};
        v.q_stride = in.q_stride ? in.q_stride : (size_t)p->M;
        v.line_act = c.line_act;
        v.act_ptr = c.act_ptr;
        v.act_node = c.act_node;
        v.k = c.k;
        v.w = PP::w(c);
        v.q = q;
        v.coef = coef;
        return v;
    };
    ra.dip = view(p->dip, in.q_dip, in.c_dip);
    ra.mono = view(p->mono, in.q_mono, in.c_mono);
    ra.grid = in.grid;
    ra.cg = in.c_grid;
    ra.grid_stride = (size_t)p->nlines * n;
    ra.spec = spec;
    ra.spec_stride = sstride;
    ra.P = p->P;
    ra.tw = PP::tw(p);
    const int G = row_lines_per_block<R>(n);
    stage_mark(p, stage++, "spread+fft_x", st);
    if (ra.nproc > 0) launch_row_fwd<R>(n, dim3((ra.nproc + G - 1) / G, nrhs), st, ra);

    // ---- columns
    const int C = col_width<R>(n);
    const int ngrp = (p->W + C - 1) / C;
    ColArgs<R> ca{};
    ca.spec = spec;
    ca.rhs_stride = sstride;
    ca.width = p->W;
    ca.tw = PP::tw(p);
    ca.s2 = PP::s2(p);
    ca.alpha = (R)p->alpha;
    ca.norm = (R)(2.0 / ((double)p->nlines * (double)n));
    if (p->dim == 2) {
        ca.outer_list = nullptr;
        ca.outer_stride = 0;
        ca.elem_stride = p->P;
        ca.lmask = dense_in ? nullptr : p->spread_line_mask;
        ca.lm_outer = 0; ca.lm_stride = 1;
        ca.smask = dense_out ? nullptr : p->gather_line_mask;
        ca.sm_outer = 0; ca.sm_stride = 1;
        ca.dim3 = 0;
        stage_mark(p, stage++, "fft_y+symbol", st);
        launch_col<R, 1>(n, dim3(ngrp, 1, nrhs), st, ca);
    } else {
        // y forward over planes that hold forcing
        ColArgs<R> y1 = ca;
        y1.outer_list = dense_in ? nullptr : p->spread_planes;
        y1.outer_stride = (size_t)n * p->P;
        y1.elem_stride = p->P;
        y1.lmask = dense_in ? nullptr : p->spread_line_mask;
        y1.lm_outer = n; y1.lm_stride = 1;
        y1.smask = nullptr;
        const int ny1 = dense_in ? n : p->n_spread_planes;
        stage_mark(p, stage++, "fft_y", st);
        if (ny1 > 0) launch_col<R, 0>(n, dim3(ngrp, ny1, nrhs), st, y1);
        // z forward, symbol, z inverse over every (kx, ky)
        ColArgs<R> z = ca;
        z.outer_list = nullptr;
        z.outer_stride = p->P;
        z.elem_stride = (size_t)n * p->P;
        z.lmask = dense_in ? nullptr : p->spread_plane_mask;
        z.lm_outer = 0; z.lm_stride = 1;
        z.smask = dense_out ? nullptr : p->gather_plane_mask;
        z.sm_outer = 0; z.sm_stride = 1;
        z.dim3 = 1;
        stage_mark(p, stage++, "fft_z+symbol", st);
        launch_col<R, 1>(n, dim3(ngrp, n, nrhs), st, z);
        // y inverse over planes something is read from
        ColArgs<R> y2 = ca;
        y2.outer_list = dense_out ? nullptr : p->gather_planes;
        y2.outer_stride = (size_t)n * p->P;
        y2.elem_stride = p->P;
        y2.lmask = nullptr;
        y2.smask = dense_out ? nullptr : p->gather_line_mask;
        y2.sm_outer = n; y2.sm_stride = 1;
        const int ny2 = dense_out ? n : p->n_gather_planes;
        stage_mark(p, stage++, "ifft_y", st);
        if (ny2 > 0) launch_col<R, 2>(n, dim3(ngrp, ny2, nrhs), st, y2);
    }

    // ---- row_inv
    RowInvArgs<R> ia{};
    ia.lines = dense_out ? nullptr : p->gather_lines;
    ia.nproc = dense_out ? p->nlines : p->n_gather_lines;
    ia.spec = spec;
    ia.spec_stride = sstride;
    ia.P = p->P;
    ia.tw = PP::tw(p);
    ia.u = out.u;
    ia.u_stride = (size_t)p->nlines * n;
    ia.line_start = p->line_start;
    ia.cell = p->cell;
    ia.taps = PP::taps(p);
    ia.part = reinterpret_cast<R*>(p->ws.part);
    ia.part_stride = (size_t)p->M * p->gpp;
    ia.M = p->M;
    ia.dim = p->dim;
    stage_mark(p, stage++, dense_out ? "ifft_x" : "ifft_x+interp", st);
    if (dense_out) {
        launch_row_inv<R, 1>(n, dim3((ia.nproc + G - 1) / G, nrhs), st, ia);
    } else {
        if (ia.nproc > 0) launch_row_inv<R, 0>(n, dim3((ia.nproc + G - 1) / G, nrhs), st, ia);
        stage_mark(p, stage++, "finish", st);
        FinishArgs fa{};
        fa.perm = p->perm;
        fa.M = p->M;
        fa.gpp = p->gpp;
        fa.part_stride = ia.part_stride;
        fa.out = out.out;
        fa.out_stride = out.out_stride ? out.out_stride : (size_t)p->M;
        fa.cA = out.cA;
        fa.in = out.in;
        fa.in_stride = out.in_stride ? out.in_stride : (size_t)p->M;
        fa.cB = out.cB;
        fa.in2 = out.in2;
        fa.in2_stride = out.in2_stride ? out.in2_stride : (size_t)p->M;
        fa.cC = out.cC;
        hipLaunchKernelGGL((k_finish<R>), dim3((p->M + 255) / 256, nrhs), dim3(256), 0, st,
                           reinterpret_cast<const R*>(p->ws.part), fa);
    }
    stage_mark(p, stage++, nullptr, st);
    IBDL_HIP_TRY(hipGetLastError());
}

}  // namespace ibdl
