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
#include <hip/hip_ext.h>

#include <algorithm>

#include <memory>
#include <type_traits>
#include <vector>

#include "fft.h"
#include "plan.h"

namespace ibdl {

constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int pow2_floor(int a) {
    int p = 1;
    while (2 * p <= a) p *= 2;
    return p;
}
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int rup64(int x) { return (x + 63) / 64 * 64; }

// Tile parameters (compile-time; overridable for tuning builds).
#ifndef IBDL_RMAX_F32
#define IBDL_RMAX_F32 16
#endif
#ifndef IBDL_RMAX_F64
#define IBDL_RMAX_F64 16
#endif
#ifndef IBDL_COLB_F32
#define IBDL_COLB_F32 64
#endif
#ifndef IBDL_COLB_F64
#define IBDL_COLB_F64 64
#endif
#ifndef IBDL_COL_LDS
#define IBDL_COL_LDS 65536
#endif
#ifndef IBDL_TWL_FULL_BYTES
#define IBDL_TWL_FULL_BYTES 8192  // largest twiddle table held whole in LDS
#endif
#ifndef IBDL_ROW_ELEMS
#define IBDL_ROW_ELEMS 2048
#endif

// Largest in-register DFT per precision (register budget).
template <typename R>
struct RMax { static constexpr int value = sizeof(R) == 4 ? IBDL_RMAX_F32 : IBDL_RMAX_F64; };

// Column-group width: C adjacent complex columns are read per row.
template <typename R>
struct ColBytes { static constexpr int value = sizeof(R) == 4 ? IBDL_COLB_F32 : IBDL_COLB_F64; };

// smallest p >= need with p = d (mod m): lines p elements apart start d elements
// (d * element bytes / 4 banks) apart in the LDS banks
constexpr int staggered_pitch(int need, int m, int d) {
    int p = need;
    while (p % m != d % m) ++p;
    return p;
}

// Column swizzle of the row transforms' LDS rows: XorRows generator M_b for row bit b
// (E: complex element bytes, W: columns per row, a power of two >= 8).
// The LDS has 64 banks of 4 bytes (S = 256 / E elements per bank row, rho = S / W
// rows of a block per bank row) and serves one instruction in phases: 16-byte reads
// in four phases of 16 lanes, lanes {0-3, 12-15, 20-27} and {4-11, 16-19, 28-31}
// and the same sets plus 32; 16-byte writes in eight phases of 8 consecutive lanes;
// 8-byte reads in two phases of 32 and 8-byte writes in four of 16.  Within a phase
// two lanes at different addresses in one bank take a cycle each.  The accesses
// that meet in one phase:
//  * transform stages: consecutive lanes take consecutive columns of a row, the
//    next row for the next W lanes;
//  * split steps (tile order, K = 64 / E consecutive rows per column, the next
//    columns in the next lanes): E = 16: the K = 4 rows of columns {0,3,5,6} (or
//    {1,2,4,7}, plus 8) meet in a read phase, which needs the four rows in four
//    cosets of that set (generators 2 and 12 of row bits 0 and 1; the read of row
//    L - k pairs odd and even rows, so bit 3 ^ bit 2 of g is the same for all
//    rows, and the writes of two adjacent columns need g != g' ^ 1: 2 and 12
//    meet all three);  E = 8: the K = 8 rows of 4 adjacent columns meet in a read
//    phase, rows of one bank half (rho = 2) or of a whole bank row, in cosets of
//    {0, 1, 2, 3}: generators 4, 8, 16 for the row bits above those that pick the
//    bank part;
//  * grid rows (x consecutive in the lanes, x / 2 the row, one column): eight or
//    more consecutive rows in one column, spread by generators that keep the
//    cosets above (3 for E = 16; 1 and 2 for E = 8).
constexpr int row_swizzle_gen(int E, int W, int b) {
    const int rho = (256 / E) / W > 1 ? (256 / E) / W : 1;
    int lr = 0;
    while ((1 << lr) < rho) ++lr;
    if (E == 16) {
        const int g1[5] = {2, 12, 3, 0, 0};  // one block row per bank row (or more)
        const int g2[5] = {0, 2, 3, 0, 0};   // two block rows per bank row
        const int m = rho == 1 ? g1[b] : rho == 2 ? g2[b] : 0;
        return m < W ? m : 0;
    }
    if (b < 3) {
        if (b < lr) return 0;
        const int m = 4 << (b - lr);
        return m < W ? m : 0;
    }
    const int m = b == 3 ? 1 : 2;
    return m < W ? m : 0;
}
template <int E, int W>
using RowSwizzle = XorRows<W, row_swizzle_gen(E, W, 0), row_swizzle_gen(E, W, 1), row_swizzle_gen(E, W, 2),
                           row_swizzle_gen(E, W, 3), row_swizzle_gen(E, W, 4)>;

// Row passes: a block transforms G lines of each of RB right-hand sides (GB lines
// in all); the right-hand sides of a block share the spread and interpolation tables.
// Variants V (chosen per configuration by the autotuner): RB = 1, 2, 4 with as
// many lines as IBDL_ROW_ELEMS elements allow, and one line of one right-hand
// side per block (most blocks, for launches with few right-hand sides).
constexpr int kRowVars = 4;
constexpr int kRowVarRB[kRowVars] = {1, 2, 4, 1};
constexpr int kRowVarG[kRowVars] = {0, 0, 0, 1};
// the one-line shape is built for FP32 only (in FP64 it spills registers)
template <typename R>
constexpr int row_vars() { return sizeof(R) == 4 ? kRowVars : 3; }
template <typename R, int N, int V = 0>
struct RowCfg {
    static constexpr int RB = kRowVarRB[V];                                   // rhs per block
    static constexpr int L = N / 2;                                           // complex length
    static constexpr int G = kRowVarG[V] > 0 ? kRowVarG[V]                    // lines per rhs
                                             : imax(1, imin(64, IBDL_ROW_ELEMS / L) / RB);
    static constexpr int GB = G * RB;                                         // lines per block
    static constexpr int T = imax(kRowVarG[V] > 0 ? 64 : 256, fft_threads<L, GB, RMax<R>::value>());
    // LDS rows of the block's lines (row k holds element k of every line):
    // power-of-two sizes with at least 8 lines: column-swizzled rows (RowSwizzle),
    // the inverse's input rows X[0..L] in the same layout (SWZ);
    // else rows narrower than the 64 four-byte banks: padded rows (PadRows) and the
    // row-inverse input lines staggered (line-major, pitch XP), so that one
    // half-wave's accesses spread over distinct banks
    static constexpr bool SWZ = is_pow2(GB) && GB >= 8 && is_pow2(L);
    static constexpr bool NARROW = GB * 2 * (int)sizeof(R) < 256;
    static constexpr int PS = !SWZ && NARROW ? first_radix_shift<L, RMax<R>::value>() : 0;
    using LAY = std::conditional_t<SWZ, RowSwizzle<2 * (int)sizeof(R), GB>, PadRows<GB, PS>>;
    static constexpr int ROWS = LAY::rows(L);
    // lanes served per LDS cycle: 256 bytes of elements; consecutive lines start
    // (that many lanes / GB) elements apart in the banks
    static constexpr int XP =
        NARROW && GB > 1 ? staggered_pitch(L + 1, 128 / (int)sizeof(R), 128 / (int)sizeof(R) / GB) : L + 1;
    // element X[k] of block line l of the inverse's input, and the elements its
    // block holds in LDS (input rows and transform rows share the storage)
    __device__ __forceinline__ static int xidx(int k, int l) { return SWZ ? LAY::idx(k, l) : l * XP + k; }
    static constexpr int SIN = SWZ ? (L + 1) * GB : imax(XP, ROWS) * GB;
};
template <typename R, int N>
struct ColCfg {
    // at most IBDL_COL_LDS bytes of LDS for the block's lines, a power of two columns
    static constexpr int C = pow2_floor(imax(1, imin(ColBytes<R>::value / (2 * (int)sizeof(R)),
                                                     IBDL_COL_LDS / (N * 2 * (int)sizeof(R)))));
    static constexpr int T = fft_threads<N, C, RMax<R>::value>();
};

// Half-spectrum layout in column tiles (complex elements, one right-hand side):
// element (line, kx), line = y (2-D) or z*n + y (3-D), kx in [0, n/2], is at
//   (line / n) * NT*n*C + (kx / C) * n*C + (line % n) * C + kx % C,
// NT = ceil((n/2+1)/C) tiles of C columns; a tile of one plane is n*C contiguous
// elements, so a column transform reads and writes contiguous memory.
template <typename R, int N>
struct Tiles {
    static constexpr int C = ColCfg<R, N>::C;
    static constexpr int NT = (N / 2 + 1 + C - 1) / C;
    static constexpr size_t PLANE = (size_t)NT * N * C;
    __device__ __forceinline__ static size_t idx(int line, int kx) {
        return (size_t)(line / N) * PLANE + (size_t)(kx / C) * (N * C) + (size_t)(line % N) * C + (kx % C);
    }
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
    const uint32_t* s;   // sorted position of each entry's point (index of qf)
    const R* w;
    uint32_t nnz;        // entries of k and w (nnz * sizeof(double) < 2^31)
    const double* q;     // q + rhs * q_stride + it * q_jstride: strengths of one right-hand side
    const R* qf;         // or null: the same strengths in R, [rhs / 4][sorted point][rhs % 4]
    int M;
    size_t q_stride;
    size_t q_jstride;    // offset per iteration index (Krylov basis vectors), else 0
    double coef;
};

template <typename R>
struct RowFwdArgs {
    const int32_t* skip;   // per-rhs flags (stride 4) or null: a set flag skips that rhs
    const int32_t* lines;  // line list or null (identity)
    int nproc;
    int nblk;              // line blocks per right-hand side
    int M;
    CsrView<R> dip, mono;
    const double* grid;    // [nrhs][n^dim] or null
    double cg;
    size_t grid_stride;
    cplx<R>* spec;
    size_t spec_stride;
    int P;
    const cplx<R>* tw;
    int nrhs;
    uint8_t* lnz;          // grid-forcing passes: per rhs (stride lnz_rhs), 1 for lines written
    size_t lnz_rhs;
};

template <typename R>
struct ColArgs {
    const int32_t* skip;
    cplx<R>* spec;
    size_t rhs_stride;
    const int32_t* outer_list;
    size_t tile_stride;   // between tiles
    size_t outer_stride;  // between outer indices (plane z, or a block of K rows)
    size_t es;            // between consecutive elements of a line (C in K == 1 passes)
    int width;            // n/2 + 1 columns
    const uint8_t* lmask;
    int lm_outer, lm_stride;
    size_t lm_rhs;        // per right-hand side (masks written by the previous pass), else 0
    const uint8_t* smask;
    int sm_outer, sm_stride;
    uint8_t* onz;         // 3-D y pass of a grid-forcing pass: per rhs (stride onz_rhs), 1 for
    size_t onz_rhs;       // the planes it writes; a plane whose lines are all unwritten is skipped
    const cplx<R>* tw;
    const R* s2;
    R alpha;
    R norm;
    const R* sym;         // 2-D FP32: norm / lambda per element in tile layout ([tile][row][C])
    int nouter;           // outer indices per right-hand side
    int nrhs;
};

template <typename R>
struct RowInvArgs {
    const int32_t* skip;
    const int32_t* lines;
    int nproc;
    int nblk;
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
    int nrhs;
};

// ------------------------------------------------------------ jobs
// A launch covers one job (arguments by value) or many jobs of the same size
// (arguments from a device table; job j owns blocks start[j] .. start[j+1]-1).
template <class A>
struct Jobs {
    const A* list;
    const int* start;     // n + 1 entries
    int n;
    const int32_t* itp;   // base of the iteration index in device memory (added to the
                          // launch argument), or null: the launch argument alone
};
__device__ __forceinline__ int job_of(const int* start, int n, int b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}
#define IBDL_JOB_ENTRY(BODY, A, a0, js, it)                          \
    const int it_ = (js.itp ? *js.itp : 0) + it;                      \
    if constexpr (MULTI) {                                            \
        const int j_ = job_of(js.start, js.n, (int)blockIdx.x);       \
        BODY(js.list[j_], (int)blockIdx.x - js.start[j_], it_);       \
    } else {                                                          \
        BODY(a0, (int)blockIdx.x, it_);                               \
    }

// ------------------------------------------------------------ strength packing
// qf[g][s][rr] = (R) q[(4g + rr) * q_stride + it * q_jstride + perm[s]], 0 past
// nrhs: the four right-hand sides of a group sit in one 16- (FP32) or 32-byte
// (FP64) segment, so the spread's adjacent lanes of one node (its right-hand
// sides) read one cache line per entry; the points go in sorted (cell) order, so
// the entries of nearby nodes, which come from the same few cells, read nearby
// segments
template <typename R>
struct PackArgs {
    const double* q;
    size_t q_stride, q_jstride;
    int M, nrhs;
    int nkb;  // blocks of 256 points per group
    const uint32_t* perm;  // caller index of each sorted position
    R* qf;
};
template <typename R>
__device__ __forceinline__ void pack_body(const PackArgs<R>& a, int lb, int it) {
    const int g = lb / a.nkb;
    const int s = (lb % a.nkb) * 256 + (int)threadIdx.x;
    if (s >= a.M) return;
    const int k = (int)a.perm[s];
    R* out = a.qf + ((size_t)g * a.M + s) * 4;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int r = 4 * g + rr;
        out[rr] = r < a.nrhs ? (R)a.q[(size_t)r * a.q_stride + (size_t)it * a.q_jstride + k] : R(0);
    }
}
template <typename R, bool MULTI>
__global__ __launch_bounds__(256) void k_pack(PackArgs<R> a0, Jobs<PackArgs<R>> js, int it) {
    IBDL_JOB_ENTRY(pack_body<R>, PackArgs<R>, a0, js, it)
}

// ------------------------------------------------------------ spread phase
// Adds coef * (sum_e w_e q[k_e]) into the LDS lines for every active node of
// the block's lines, for each of the block's right-hand sides (rhs_s[rr] >= 0):
// the entries of a node are loaded once for all of them.  Each node is written
// by exactly one thread, its entries summed in their stored order.  la[g] is the
// first active node of line g and rs the prefix sums of the lines' node counts.
template <typename R, int N, int G, int RB, int T, class LAY>
__device__ __forceinline__ void spread_phase(R* sr, const CsrView<R>& c, int it, const int* la, const int* rs,
                                             const int* rhs_s) {
    constexpr int GB = G * RB;
    const int total = rs[G];
    // work item f: node f / RB for the block's right-hand side f % RB; the RB items of
    // a node sit in adjacent lanes, so their entry loads are one request per wavefront
    for (int f = threadIdx.x; f < total * RB; f += T) {
        const int rr = f % RB, nf = f / RB;
        const int r = rhs_s[rr];
        if (r < 0) continue;
        int lo = 0, hi = G;  // find g with rs[g] <= nf < rs[g+1]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (rs[mid] <= nf) lo = mid; else hi = mid;
        }
        const int g = lo;
        const int a = la[g] + (nf - rs[g]);
        const int x = (int)(c.act_node[a] % (uint32_t)N);
        const double* q = c.q + (size_t)r * c.q_stride + (size_t)it * c.q_jstride;
        // packed strengths (the same values the sum rounds q to): the lanes of a
        // node's right-hand sides read one segment per entry
        const R* qf = c.qf ? c.qf + (size_t)(r >> 2) * c.M * 4 + (r & 3) : nullptr;
        Acc<R> acc;
        const int e1 = c.act_ptr[a + 1];
        // entries in groups of 8 through buffer descriptors over k and w (one offset per
        // group, the entries at immediate offsets from it): every load of a group is
        // issued before any is used; entries past the node's last belong to the next
        // node or lie past the arrays (read as 0) and enter with weight 0 (adding
        // 0 * q leaves both parts of the sum exactly as they were), so the group has
        // no branch
        // packed strengths are indexed by sorted position, the caller's by caller index
        const __amdgpu_buffer_rsrc_t rk = buf_rsrc(qf ? c.s : c.k, c.nnz * 4u);
        const __amdgpu_buffer_rsrc_t rw = buf_rsrc(c.w, c.nnz * (uint32_t)sizeof(R));
        for (int e = c.act_ptr[a]; e < e1; e += 8) {
            const int cnt = e1 - e;
            uint32_t kk[8];
            R ww[8];
            R qq[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                kk[u] = __builtin_amdgcn_raw_buffer_load_b32(rk, e * 4 + u * 4, 0, 0);
                const R wv = BufScalar<R>::load(rw, e * (int)sizeof(R) + u * (int)sizeof(R));
                ww[u] = u < cnt ? wv : R(0);
            }
            if (qf) {
#pragma unroll
                for (int u = 0; u < 8; ++u) qq[u] = (R)qf[(size_t)kk[u] * 4];
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) qq[u] = (R)q[kk[u]];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc.add(ww[u], qq[u]);
        }
        R& node = sr[2 * LAY::idx(x >> 1, rr * G + g) + (x & 1)];
        node = fmac((R)c.coef, acc.value(), node);
    }
    __syncthreads();
}

// ------------------------------------------------------------ row_fwd
// Block lb covers lines [b G, b G + G) of the line list for the right-hand sides
// rg RB .. rg RB + RB - 1 (b = lb % nblk, rg = lb / nblk); LDS line rr G + g holds
// line g of the rr-th of them.
template <typename R, int N, int V>
__device__ __forceinline__ void row_fwd_body(const RowFwdArgs<R>& a, int lb, int it) {
    using CF = RowCfg<R, N, V>;
    constexpr int RB = CF::RB, L = CF::L, G = CF::G, GB = CF::GB, T = CF::T;
    using LAY = typename CF::LAY;
    __shared__ cplx<R> s[CF::ROWS * GB];
    __shared__ int rs[2][G + 1], la[2][G];
    __shared__ int lines_s[G], rhs_s[RB];
    __shared__ int nzl[GB];  // grid-forcing passes: 1 for block lines with a nonzero grid row
    using TWL = TwLds<R, N, (N * 2 * (int)sizeof(R) <= IBDL_TWL_FULL_BYTES)>;
    __shared__ cplx<R> twl[TWL::SIZE];
    R* sr = reinterpret_cast<R*>(s);
    const int rg = lb / a.nblk;
    const int first = (lb % a.nblk) * G;
    // every table load of the block at once: skip flags, twiddles, line ids and
    // the lines' active-node ranges of both spread matrices
    int live = 0, rv[RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
        const int r = rg * RB + rr;
        rv[rr] = (r < a.nrhs && !(a.skip && a.skip[4 * r])) ? r : -1;
        live |= rv[rr] >= 0;
    }
    const auto tw = TWL::template load<T>(twl, a.tw);
    if (threadIdx.x < G) {
        const int g = threadIdx.x;
        const int li = first + g;
        int line = -1, c0 = 0, c1 = 0, m0 = 0, m1 = 0;
        if (li < a.nproc) {
            line = a.lines ? a.lines[li] : li;
            if (a.dip.q) {
                c0 = a.dip.line_act[line];
                c1 = a.dip.line_act[line + 1];
            }
            if (a.mono.q) {
                m0 = a.mono.line_act[line];
                m1 = a.mono.line_act[line + 1];
            }
        }
        lines_s[g] = line;
        la[0][g] = c0;
        rs[0][g + 1] = c1 - c0;
        la[1][g] = m0;
        rs[1][g + 1] = m1 - m0;
    }
    if (!live) return;
    if (threadIdx.x < RB) rhs_s[threadIdx.x] = rv[threadIdx.x];
    if (threadIdx.x < GB) nzl[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < CF::ROWS * GB; i += T) s[i] = cplx<R>{R(0), R(0)};
    __syncthreads();
    if (threadIdx.x < 2) {
        int* r = rs[threadIdx.x];
        r[0] = 0;
        for (int g = 1; g <= G; ++g) r[g] += r[g - 1];
    }
    if (a.grid) {
        // every load of the block's grid rows is issued before the first is stored
        constexpr int PER = (N * GB + T - 1) / T;
        double v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int id = threadIdx.x + u * T;
            const int l = id / N, x = id % N;
            const int line = id < N * GB ? lines_s[l % G] : -1;
            const int r = id < N * GB ? rhs_s[l / G] : -1;
            v[u] = (line >= 0 && r >= 0) ? a.grid[(size_t)r * a.grid_stride + (size_t)line * N + x] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int id = threadIdx.x + u * T;
            const int l = id / N, x = id % N;
            if (id < N * GB) {
                sr[2 * LAY::idx(x >> 1, l) + (x & 1)] = (R)(a.cg * v[u]);
                if (v[u] != 0.0) nzl[l] = 1;  // every writer stores the same value
            }
        }
    }
    __syncthreads();
    if (a.dip.q) spread_phase<R, N, G, RB, T, LAY>(sr, a.dip, it, la[0], rs[0], rhs_s);
    if (a.mono.q) spread_phase<R, N, G, RB, T, LAY>(sr, a.mono, it, la[1], rs[1], rhs_s);

    // grid-forcing passes: a line with a zero grid row and no spread entries has a
    // zero spectrum; it is flagged 0 for the column passes, which read it as zero,
    // and not stored; a block all of whose lines are zero skips its transform
    if (a.lnz) {
        int nz = 0;
        if (threadIdx.x < GB) {
            const int l = threadIdx.x, g = l % G;
            const int line = lines_s[g], r = rhs_s[l / G];
            nz = nzl[l] | (a.dip.q && rs[0][g + 1] > rs[0][g]) | (a.mono.q && rs[1][g + 1] > rs[1][g]);
            nzl[l] = nz;
            if (line >= 0 && r >= 0) a.lnz[(size_t)r * a.lnz_rhs + line] = (uint8_t)nz;
        }
        if (!__syncthreads_or(nz)) return;
    }
    run_fft<R, L, GB, T, N, -1, LAY>(s, tw, LdsLoad<R, LAY>{s}, LdsStore<R, LAY>{s},
                                    FwdRadices<L, RMax<R>::value>{});
    __syncthreads();

    // split step: X[k] = (Z_k + conj Z_{L-k})/2 - i W_N^k (Z_k - conj Z_{L-k})/2, k = 0..L,
    // written in tile order so that consecutive threads store consecutive addresses
    using TL = Tiles<R, N>;
    constexpr int C = TL::C;
    for (int id = threadIdx.x; id < TL::NT * GB * C; id += T) {
        const int t = id / (GB * C), rem = id % (GB * C);
        const int l = rem / C, c = rem % C;
        const int k = t * C + c;
        const int line = lines_s[l % G];
        const int r = rhs_s[l / G];
        if (k > L || line < 0 || r < 0 || (a.lnz && !nzl[l])) continue;
        const cplx<R> zk = s[LAY::idx(k % L, l)];
        const cplx<R> zm = s[LAY::idx((L - k) % L, l)];
        const cplx<R> e = cscale(cadd(zk, cconj(zm)), R(0.5));
        const cplx<R> d = cscale(csub(zk, cconj(zm)), R(0.5));
        a.spec[(size_t)r * a.spec_stride + TL::idx(line, k)] = cadd(e, cmul(tw.get(k), cmul_si<-1>(d)));
    }
}
template <typename R, int N, int V, bool MULTI>
__global__ __launch_bounds__((RowCfg<R, N, V>::T)) void k_row_fwd(RowFwdArgs<R> a0, Jobs<RowFwdArgs<R>> js,
                                                                   int it) {
    IBDL_JOB_ENTRY((row_fwd_body<R, N, V>), RowFwdArgs<R>, a0, js, it)
}

// ------------------------------------------------------------ col
// A block transforms K*C lines of length N: element i of line l at
// base + i * es + l, with the C columns of tile t (kx = t*C + l % C) and, for
// K > 1, K consecutive y-rows (ky = o*K + l / C) of the z-transform.
// Element i of line l through the block's buffer descriptor (esb: bytes between
// consecutive elements of a line, below 2^24; ES > 0: the same as a compile-time
// element count): lines whose column l % C is past the spectrum's width
// (l % C >= vcols) and rows outside the row set map to an offset of 2^31 or more,
// past every range (read as zero, store dropped), with no branch.  The row set
// is held in LDS as one byte per row, 0 (in) or 0x80 (out), which lands on bit 31;
// in-range offsets stay below 2^31.
template <typename R, int C, int ES>
__device__ __forceinline__ int col_offset(int i, int l, int esb, int vcols, const uint8_t* m) {
    const unsigned lo = (l % C) < vcols ? (unsigned)(l * (int)sizeof(cplx<R>)) : 0x80000000u;
    const unsigned row = ES > 0 ? (unsigned)i * (unsigned)(ES * (int)sizeof(cplx<R>))
                                : __umul24((unsigned)i, (unsigned)esb);
    return (int)((row + lo) | ((unsigned)m[i] << 24));
}
template <typename R, int C, int ES>
struct ColLoad {
    __amdgpu_buffer_rsrc_t rs;
    int esb, vcols;
    const uint8_t* m;  // LDS row set (0 in, 0x80 out)
    __device__ __forceinline__ cplx<R> operator()(int i, int l) const {
        return BufIO<R>::load(rs, col_offset<R, C, ES>(i, l, esb, vcols, m));
    }
};
template <typename R, int C, int ES>
struct ColStore {
    __amdgpu_buffer_rsrc_t rs;
    int esb, vcols;
    const uint8_t* m;
    __device__ __forceinline__ void operator()(int i, int l, cplx<R> v) const {
        BufIO<R>::store(rs, col_offset<R, C, ES>(i, l, esb, vcols, m), v);
    }
};
// 1/x: hardware reciprocal (about 1 ulp) in FP32, exact division in FP64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
// LDS store that multiplies by norm / lambda(k), lambda = -(sum_d (4/h^2) sin^2(pi k_d/n)) - alpha:
// srow[i] is the line-axis term, scol[l] the other axes plus alpha (-1: invalid line)
template <typename R, int LC>
struct SymStore {
    cplx<R>* s;
    const R* srow;
    const R* scol;
    R norm;
    __device__ __forceinline__ void operator()(int i, int l, cplx<R> v) const {
        const R cc = scol[l];
        const R lam = srow[i] + cc;
        const R sig = (cc >= R(0) && lam != R(0)) ? -norm * recip(lam) : R(0);
        s[i * LC + l] = cscale(v, sig);
    }
};

// LDS store that multiplies output slot k by the inverse symbol prefetched for it
template <typename R, int LC>
struct SymTabStore {
    cplx<R>* s;
    const R* sig;  // the thread's prefetched values, one per output slot
};
template <typename R, int LC>
__device__ __forceinline__ void store_out(SymTabStore<R, LC>& st, int i, int l, cplx<R> v, int k) {
    st.s[i * LC + l] = cscale(v, st.sig[k]);
}

// A column block covers K y-rows (3-D z transform: K > 1) of its tile's C columns.
template <typename R, int N, int K>
struct ColK {
    static constexpr int C = ColCfg<R, N>::C;
    static constexpr int LC = K * C;
    static constexpr int T = fft_threads<N, LC, RMax<R>::value>();
};

// MODE 0: forward; 1: forward, times inverse symbol, inverse; 2: inverse.
template <typename R, int N, int MODE, int K>
__device__ __forceinline__ void col_body(const ColArgs<R>& a, int lb, int) {
    using CK = ColK<R, N, K>;
    constexpr int C = CK::C, LC = CK::LC, T = CK::T, RM = RMax<R>::value;
    constexpr int NT = (N / 2 + 1 + C - 1) / C;
    __shared__ cplx<R> s[N * LC];
    __shared__ uint8_t lmask[N], smask[N];
    __shared__ R srow[MODE == 1 ? N : 1];
    __shared__ R scol[MODE == 1 ? LC : 1];
    // the full twiddle table in LDS where it keeps two blocks per compute unit
    using TWL = TwLds<R, N, (N * 2 * (int)sizeof(R) <= IBDL_TWL_FULL_BYTES)>;
    __shared__ cplx<R> twl[TWL::SIZE];
    // A last tile that holds only the column kx = n/2 is transformed alone (below),
    // and its blocks come after all full tiles so that the full tiles spread
    // evenly over the compute units.
    constexpr bool NYQ = K == 1 && (N / 2) % C == 0;
    constexpr int NTF = NYQ ? NT - 1 : NT;
    const int pairs = a.nouter * a.nrhs;
    int t, pr;
    if (lb < NTF * pairs) {
        t = lb % NTF;
        pr = lb / NTF;
    } else {
        t = NT - 1;
        pr = lb - NTF * pairs;
    }
    const int oi = pr % a.nouter;
    const int rhs = pr / a.nouter;
    const int o = a.outer_list ? a.outer_list[oi] : oi;
    // every table load of the block at once: skip flag, twiddles, row masks, symbol terms
    const int32_t skipv = a.skip ? a.skip[4 * rhs] : 0;
    const auto tw = TWL::template load<T>(twl, a.tw);
    constexpr int PN = (N + T - 1) / T, PL = (LC + T - 1) / T;
    uint8_t lmv[PN], smv[PN];
    R s2v[PN];
#pragma unroll
    for (int u = 0; u < PN; ++u) {
        const int i = threadIdx.x + u * T;
        if (i < N) {
            lmv[u] = a.lmask ? a.lmask[(size_t)rhs * a.lm_rhs + o * a.lm_outer + i * a.lm_stride] : 1;
            smv[u] = a.smask ? a.smask[o * a.sm_outer + i * a.sm_stride] : 1;
            if constexpr (MODE == 1) s2v[u] = a.s2[i];
        }
    }
    R scv[PL];
#pragma unroll
    for (int u = 0; u < PL; ++u) {
        const int l = threadIdx.x + u * T;
        if (l < LC) {
            const int kx = t * C + l % C;
            if constexpr (MODE == 1)
                scv[u] = kx < a.width ? a.s2[kx] + (K > 1 ? a.s2[o * K + l / C] : R(0)) + a.alpha : R(-1);
        }
    }
    // 2-D FP32 (K == 1, MODE 1): the inverse symbol of every output of the last
    // forward stage comes from the plan's table, loaded here with the other tables
    // (not at n = 2048, whose kernel holds 121 VGPRs without the prefetched values
    // and would lose its second block per compute unit past 128)
    constexpr bool SYMT = MODE == 1 && K == 1 && sizeof(R) == 4 && N < 2048;
    constexpr int RL = last_radix<N, RM>(), NBL = N / RL, TOTL = NBL * LC, PERL = (TOTL + T - 1) / T;
    R sigv[SYMT ? PERL * RL : 1];
    if constexpr (SYMT) {
        // rows past N (threads beyond the last stage's butterflies) read 0 and are not used
        const __amdgpu_buffer_rsrc_t rsym =
            buf_rsrc(a.sym + (size_t)t * N * C, (uint32_t)(N * C * (int)sizeof(R)));
#pragma unroll
        for (int b = 0; b < PERL; ++b) {
            const int id = threadIdx.x + b * T;
            const int c = id % LC, j = id / LC;
#pragma unroll
            for (int r = 0; r < RL; ++r)
                sigv[b * RL + r] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                    rsym, ((j + r * NBL) * C + c) * (int)sizeof(R), 0, 0));
        }
    }
    if (skipv) return;
    if (a.onz) {
        // a plane none of whose lines was written is zero: its transform is zero too
        int any = 0;
#pragma unroll
        for (int u = 0; u < PN; ++u) any |= (threadIdx.x + u * T < N) && lmv[u];
        any = __syncthreads_or(any);
        if (threadIdx.x == 0) a.onz[(size_t)rhs * a.onz_rhs + o] = (uint8_t)(any != 0);
        if (!any) return;
    }
    // the block's elements i * es + l (i < N, l < LC) from its base: at most
    // (511 * 65 * 512 * 4 + 16) * 16 bytes (3-D, n <= 512, FP64), below 2^31
    const cplx<R>* base = a.spec + (size_t)rhs * a.rhs_stride + (size_t)t * a.tile_stride + (size_t)o * a.outer_stride;
    // K == 1 passes (2-D, and the 3-D y passes) step C elements along a line
    constexpr int ES = K == 1 ? C : 0;
    const int es = K == 1 ? C : (int)a.es;
    const int esb = es * (int)sizeof(cplx<R>);
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(base, (uint32_t)(((N - 1) * es + LC) * (int)sizeof(cplx<R>)));
    const int vcols = a.width - t * C;
#pragma unroll
    for (int u = 0; u < PN; ++u) {
        const int i = threadIdx.x + u * T;
        if (i < N) {
            lmask[i] = lmv[u] ? 0 : 0x80;
            smask[i] = smv[u] ? 0 : 0x80;
            if constexpr (MODE == 1) srow[i] = s2v[u];
        }
    }
#pragma unroll
    for (int u = 0; u < PL; ++u) {
        const int l = threadIdx.x + u * T;
        if (l < LC) {
            if constexpr (MODE == 1) scol[l] = scv[u];
        }
    }
    __syncthreads();
    if constexpr (NYQ) {
        if (t == NT - 1) {
            // the last tile holds only the column kx = n/2: transform it alone
            const ColLoad<R, C, ES> ld1{rs, esb, vcols, lmask};
            const ColStore<R, C, ES> st1{rs, esb, vcols, smask};
            if constexpr (MODE == 0) {
                run_fft<R, N, 1, T, N, -1>(s, tw, ld1, st1, FwdRadices<N, RM>{});
            } else if constexpr (MODE == 2) {
                run_fft<R, N, 1, T, N, +1>(s, tw, ld1, st1, FwdRadices<N, RM>{});
            } else {
                const SymStore<R, 1> sym1{s, srow, scol, a.norm};
                run_fft<R, N, 1, T, N, -1>(s, tw, ld1, sym1, FwdRadices<N, RM>{});
                __syncthreads();
                run_fft<R, N, 1, T, N, +1>(s, tw, LdsLoad<R, PadRows<1>>{s}, st1, RevRadices<N, RM>{});
            }
            return;
        }
    }
    const ColLoad<R, C, ES> ld{rs, esb, vcols, lmask};
    const ColStore<R, C, ES> st{rs, esb, vcols, smask};
    if constexpr (MODE == 0) {
        run_fft<R, N, LC, T, N, -1>(s, tw, ld, st, FwdRadices<N, RM>{});
    } else if constexpr (MODE == 2) {
        run_fft<R, N, LC, T, N, +1>(s, tw, ld, st, FwdRadices<N, RM>{});
    } else if constexpr (SYMT) {
        static_assert(std::is_same<R, float>::value, "symbol table is FP32");
        run_fft<R, N, LC, T, N, -1>(s, tw, ld, SymTabStore<R, LC>{s, sigv}, FwdRadices<N, RM>{});
        __syncthreads();
        run_fft<R, N, LC, T, N, +1>(s, tw, LdsLoad<R, PadRows<LC>>{s}, st, RevRadices<N, RM>{});
    } else {
        const SymStore<R, LC> sym{s, srow, scol, a.norm};
        run_fft<R, N, LC, T, N, -1>(s, tw, ld, sym, FwdRadices<N, RM>{});
        __syncthreads();
        run_fft<R, N, LC, T, N, +1>(s, tw, LdsLoad<R, PadRows<LC>>{s}, st, RevRadices<N, RM>{});
    }
}
template <typename R, int N, int MODE, int K, bool MULTI>
__global__ __launch_bounds__((ColK<R, N, K>::T)) void k_col(ColArgs<R> a0, Jobs<ColArgs<R>> js, int it) {
    IBDL_JOB_ENTRY((col_body<R, N, MODE, K>), ColArgs<R>, a0, js, it)
}

// ------------------------------------------------------------ row_inv
// OUT 0: interpolation partial sums; OUT 1: grid output; OUT 2: both.  Blocks
// map to lines and right-hand sides as in row_fwd.
template <typename R, int N, int OUT, int V>
__device__ __forceinline__ void row_inv_body(const RowInvArgs<R>& a, int lb, int) {
    using CF = RowCfg<R, N, V>;
    constexpr int RB = CF::RB, L = CF::L, G = CF::G, GB = CF::GB, T = CF::T;
    using LAY = typename CF::LAY;
    // the block's spectrum rows X[0..L] (xs, at CF::xidx) are only read by the first
    // stage of the inverse transform, whose outputs (s) therefore share the storage
    __shared__ cplx<R> s[CF::SIN];
    cplx<R>* xs = s;
    using TWL = TwLds<R, N, (N * 2 * (int)sizeof(R) <= IBDL_TWL_FULL_BYTES)>;
    __shared__ cplx<R> twl[TWL::SIZE];
    __shared__ int lines_s[G], rhs_s[RB];
    R* sr = reinterpret_cast<R*>(s);
    const int rg = lb / a.nblk;
    const int first = (lb % a.nblk) * G;
    int live = 0, rv[RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
        const int r = rg * RB + rr;
        rv[rr] = (r < a.nrhs && !(a.skip && a.skip[4 * r])) ? r : -1;
        live |= rv[rr] >= 0;
    }
    const auto tw = TWL::template load<T>(twl, a.tw);
    if (threadIdx.x < G) {
        const int li = first + threadIdx.x;
        lines_s[threadIdx.x] = li < a.nproc ? (a.lines ? a.lines[li] : li) : -1;
    }
    if (!live) return;
    if (threadIdx.x < RB) rhs_s[threadIdx.x] = rv[threadIdx.x];
    __syncthreads();
    // the block's rows, read in tile order (consecutive threads, consecutive addresses),
    // and (interpolation) the sorted-point ranges of the x-lines (cy, cz), cy in y-2..y+1,
    // cz in z-2..z+1, of every line of the block
    using TL = Tiles<R, N>;
    constexpr int C = TL::C;
    __shared__ int rb[OUT != 1 ? G * 8 : 1], rc[OUT != 1 ? G * 8 : 1], roff[OUT != 1 ? G * 8 + 1 : 1];
    {
        // every load of the block's rows is issued before the first is stored
        constexpr int TOT = TL::NT * GB * C;
        constexpr int PER = (TOT + T - 1) / T;
        cplx<R> v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int id = threadIdx.x + u * T;
            const int t = id / (GB * C), rem = id % (GB * C);
            const int l = rem / C, c = rem % C;
            const int k = t * C + c;
            const int line = id < TOT ? lines_s[l % G] : -1;
            const int r = id < TOT ? rhs_s[l / G] : -1;
            v[u] = (line >= 0 && r >= 0 && k <= L) ? a.spec[(size_t)r * a.spec_stride + TL::idx(line, k)]
                                                   : cplx<R>{R(0), R(0)};
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int id = threadIdx.x + u * T;
            const int t = id / (GB * C), rem = id % (GB * C);
            const int l = rem / C, c = rem % C;
            const int k = t * C + c;
            if (id < TOT && k <= L) xs[CF::xidx(k, l)] = v[u];
        }
    }
    if constexpr (OUT != 1) {
        const int nz = a.dim == 3 ? 4 : 1;
        for (int t = threadIdx.x; t < G * 4; t += T) {
            const int g = t / 4, dz = t % 4;
            int b0 = 0, c0 = 0, b1 = 0, c1 = 0;
            const int line = lines_s[g];
            if (line >= 0 && dz < nz) {
                const int y = line % N, z = line / N;
                const int cz = a.dim == 3 ? (z - 2 + dz + N) % N : 0;
                const int pz = cz * N;
                const int lo = y - 2, hi = y + 2;
                if (lo < 0) {
                    b0 = a.line_start[pz + lo + N];
                    c0 = a.line_start[pz + N] - b0;
                    b1 = a.line_start[pz];
                    c1 = a.line_start[pz + hi] - b1;
                } else if (hi > N) {
                    b0 = a.line_start[pz + lo];
                    c0 = a.line_start[pz + N] - b0;
                    b1 = a.line_start[pz];
                    c1 = a.line_start[pz + hi - N] - b1;
                } else {
                    b0 = a.line_start[pz + lo];
                    c0 = a.line_start[pz + hi] - b0;
                }
            }
            rb[2 * t] = b0;
            rc[2 * t] = c0;
            rb[2 * t + 1] = b1;
            rc[2 * t + 1] = c1;
        }
    }
    __syncthreads();
    // interpolation: the first work item of every thread, fetched before the transform
    int pf_s = -1, pf_r = 0, pf_rr = 0;
    int pf_cell[3] = {0, 0, 0};
    R pf_tp[12];
    if constexpr (OUT != 1) {
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int r = 0; r < G * 8; ++r) {
                roff[r] = acc;
                acc += rc[r];
            }
            roff[G * 8] = acc;
        }
        __syncthreads();
        const int f = threadIdx.x / RB;
        pf_rr = threadIdx.x % RB;
        if ((int)threadIdx.x < roff[G * 8] * RB) {
            int lo = 0, hi = G * 8;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (roff[mid] <= f) lo = mid; else hi = mid;
            }
            pf_r = lo;
            pf_s = rb[lo] + (f - roff[lo]);
#pragma unroll
            for (int d = 0; d < 3; ++d) pf_cell[d] = a.cell[3 * pf_s + d];
#pragma unroll
            for (int u = 0; u < 12; ++u) pf_tp[u] = a.taps[(size_t)pf_s * 12 + u];
        }
    }
    // inverse split step: Z_k = (X_k + conj X_{L-k})/2 + i W_N^-k (X_k - conj X_{L-k})/2
    auto split = [&](int k, int l) -> cplx<R> {
        const cplx<R> xk = xs[CF::xidx(k, l)];
        const cplx<R> xm = xs[CF::xidx(L - k, l)];
        const cplx<R> e = cscale(cadd(xk, cconj(xm)), R(0.5));
        const cplx<R> d = cscale(csub(xk, cconj(xm)), R(0.5));
        return cadd(e, cmul_si<1>(cmul(cconj(tw.get(k)), d)));
    };
    run_fft<R, L, GB, T, N, +1, LAY>(s, tw, split, LdsStore<R, LAY>{s}, FwdRadices<L, RMax<R>::value>{});
    __syncthreads();

    if constexpr (OUT != 0) {
        for (int id = threadIdx.x; id < GB * N; id += T) {
            const int l = id / N, x = id % N;
            const int line = lines_s[l % G];
            const int r = rhs_s[l / G];
            if (line >= 0 && r >= 0)
                a.u[(size_t)r * a.u_stride + (size_t)line * N + x] =
                    (double)sr[2 * LAY::idx(x >> 1, l) + (x & 1)];
        }
    }
    if constexpr (OUT != 1) {
        const int gpp = a.dim == 3 ? 16 : 4;
        // work item f: point f / RB for the block's right-hand side f % RB (adjacent
        // lanes share the point's cell and taps)
        auto gather = [&](int rr8, int rr, int sidx, const int* cell, const R* tp) {
            const int r = rhs_s[rr];
            if (r < 0) return;
            const int g = rr8 / 8;
            const int line = lines_s[g];
            const int y = line % N, z = line / N;
            const int cx = cell[0], cy = cell[1];
            const int oy = (y - cy + 1 + N) % N;
            const int l = rr * G + g;
            R acc = R(0);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int x = (cx - 1 + t + N) % N;
                acc = fmac(tp[t], sr[2 * LAY::idx(x >> 1, l) + (x & 1)], acc);
            }
            acc *= tp[4 + oy];
            int o = oy;
            if (a.dim == 3) {
                const int oz = (z - cell[2] + 1 + N) % N;
                acc *= tp[8 + oz];
                o += 4 * oz;
            }
            a.part[(size_t)r * a.part_stride + (size_t)sidx * gpp + o] = acc;
        };
        if (pf_s >= 0) gather(pf_r, pf_rr, pf_s, pf_cell, pf_tp);
        const int total = roff[G * 8] * RB;
        for (int f = threadIdx.x + T; f < total; f += T) {
            const int rr = f % RB, pf = f / RB;
            int lo = 0, hi = G * 8;  // range r with roff[r] <= pf < roff[r+1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (roff[mid] <= pf) lo = mid; else hi = mid;
            }
            const int sidx = rb[lo] + (pf - roff[lo]);
            int cell[3];
            R tp[12];
#pragma unroll
            for (int d = 0; d < 3; ++d) cell[d] = a.cell[3 * sidx + d];
#pragma unroll
            for (int u = 0; u < 12; ++u) tp[u] = a.taps[(size_t)sidx * 12 + u];
            gather(lo, rr, sidx, cell, tp);
        }
    }
}
template <typename R, int N, int OUT, int V, bool MULTI>
__global__ __launch_bounds__((RowCfg<R, N, V>::T)) void k_row_inv(RowInvArgs<R> a0, Jobs<RowInvArgs<R>> js,
                                                                   int it) {
    IBDL_JOB_ENTRY((row_inv_body<R, N, OUT, V>), RowInvArgs<R>, a0, js, it)
}

// ------------------------------------------------------------ finish
struct FinishArgs {
    const int32_t* skip;
    const uint32_t* perm;
    int M, gpp;
    int nblk;             // point blocks per right-hand side
    const void* part;     // gather partials of the plan's precision
    size_t part_stride;
    double* out;          // + rhs * out_stride + it * out_jstride
    size_t out_stride, out_jstride;
    double cA;
    const double* in;
    size_t in_stride, in_jstride;
    double cB;
    const double* in2;
    size_t in2_stride;
    double cC;
    // optional: partial <out, V_i> for i < nv over each block's points (Arnoldi step)
    const double* V;
    size_t vstride_rhs;   // between right-hand sides
    int nv;               // number of basis vectors (V_i at V + i*M), plus it
    double* dots;         // [rhs][block][dstride]
    size_t dots_rhs;
    int dstride;
};

constexpr int FIN_T = 256;

template <typename R>
__device__ __forceinline__ void finish_body(const FinishArgs& f, int lb, int it) {
    const int rhs = lb / f.nblk;
    const int s = (lb % f.nblk) * FIN_T + threadIdx.x;
    // skip flag, point index and partials are loaded together
    const int32_t skipv = f.skip ? f.skip[4 * rhs] : 0;
    double v = 0.0;
    uint32_t k = 0;
    double acc = 0.0;
    if (s < f.M) {
        const R* p = reinterpret_cast<const R*>(f.part) + (size_t)rhs * f.part_stride + (size_t)s * f.gpp;
        k = f.perm[s];
        if (f.gpp == 4) {
            R pv[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) pv[o] = p[o];
#pragma unroll
            for (int o = 0; o < 4; ++o) acc += (double)pv[o];
        } else {
            R pv[16];
#pragma unroll
            for (int o = 0; o < 16; ++o) pv[o] = p[o];
#pragma unroll
            for (int o = 0; o < 16; ++o) acc += (double)pv[o];
        }
    }
    if (skipv) return;
    if (s < f.M) {
        v = f.cA * acc;
        if (f.in) v += f.cB * f.in[(size_t)rhs * f.in_stride + (size_t)it * f.in_jstride + k];
        if (f.in2) v += f.cC * f.in2[(size_t)rhs * f.in2_stride + k];
        f.out[(size_t)rhs * f.out_stride + (size_t)it * f.out_jstride + k] = v;
    }
    if (!f.V) return;
    // fixed-order block reductions of v * V_i[k], 16 basis vectors per LDS pass
    __shared__ double sh[(FIN_T / 64) * 16];
    const double* Vr = f.V + (size_t)rhs * f.vstride_rhs;
    double* d = f.dots + (size_t)rhs * f.dots_rhs + (size_t)(lb % f.nblk) * f.dstride;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int nvt = f.nv + it;
    for (int v0 = 0; v0 < nvt; v0 += 16) {
        const int nv = nvt - v0 < 16 ? nvt - v0 : 16;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (u < nv) {
                double t = s < f.M ? v * Vr[(size_t)(v0 + u) * f.M + k] : 0.0;
                for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
                if (l == 0) sh[w * 16 + u] = t;
            }
        }
        __syncthreads();
        if (threadIdx.x < nv) {
            double t = 0.0;
            for (int ww = 0; ww < FIN_T / 64; ++ww) t += sh[ww * 16 + threadIdx.x];
            d[v0 + threadIdx.x] = t;
        }
        __syncthreads();
    }
}
template <typename R, bool MULTI>
__global__ __launch_bounds__(FIN_T) void k_finish(FinishArgs a0, Jobs<FinishArgs> js, int it) {
    IBDL_JOB_ENTRY((finish_body<R>), FinishArgs, a0, js, it)
}

// ------------------------------------------------------------ dispatch
#define IBDL_SIZES(X) \
    X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048)

template <typename R>
inline int row_lines_per_block(int n, int v) {
    switch (n) {
#define IBDL_C(NN) \
    case NN: return v == 3 ? RowCfg<R, NN, 3>::G : v == 2 ? RowCfg<R, NN, 2>::G : v == 1 ? RowCfg<R, NN, 1>::G \
                                                                                      : RowCfg<R, NN, 0>::G;
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
inline int col_tiles(int n) {
    switch (n) {
#define IBDL_C(NN) case NN: return Tiles<R, NN>::NT;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
    return 1;
}
// y-rows per block of the 3-D z transform while the block's lines fit 128 KiB of LDS:
// up to 4 in FP64 and 2 in FP32.  Measured on the sphere 256^3 at 32 rhs: FP32 2 rows
// (32 KiB, four blocks per CU) 0.72 -> 0.68 ms against 4; FP64 2 rows 1.26 -> 1.35 ms
// (its 154 VGPRs hold it at two waves per SIMD either way)
#ifndef IBDL_ZROWS_MAX_F64
#define IBDL_ZROWS_MAX_F64 4
#endif
#ifndef IBDL_ZROWS_MAX_F32
#define IBDL_ZROWS_MAX_F32 2
#endif
template <typename R, int N>
struct ZRows {
    static constexpr int value =
        imax(1, imin(sizeof(R) == 4 ? IBDL_ZROWS_MAX_F32 : IBDL_ZROWS_MAX_F64,
                     131072 / (N * ColCfg<R, N>::C * 2 * (int)sizeof(R))));
};
template <typename R>
inline int z_rows(int n) {
    switch (n) {
#define IBDL_C(NN) case NN: return ZRows<R, NN>::value;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
    return 1;
}

template <class A>
struct StageTable {
    std::vector<A> args;
    std::vector<int> start{0};  // block offsets, njobs + 1 entries
    const A* dargs = nullptr;   // device copies (several jobs)
    const int* dstart = nullptr;
    void add(const A& a, int blocks) {
        args.push_back(a);
        start.push_back(start.back() + blocks);
    }
    int njobs() const { return (int)args.size(); }
    int blocks() const { return start.back(); }
    bool multi() const { return njobs() > 1; }
    Jobs<A> jobs(const int32_t* itp) const { return Jobs<A>{dargs, dstart, njobs(), itp}; }
    void upload(Arena& ar, hipStream_t st) {
        if (!multi()) return;
        dargs = reinterpret_cast<const A*>(arena_stage(ar, args.data(), args.size() * sizeof(A), st));
        dstart = reinterpret_cast<const int*>(arena_stage(ar, start.data(), start.size() * sizeof(int), st));
    }
};

template <typename R, int V, bool MULTI>
void launch_row_fwd_v(int n, int blocks, hipStream_t st, StageEv e, const RowFwdArgs<R>& a,
                      Jobs<RowFwdArgs<R>> js, int it) {
    switch (n) {
#define IBDL_C(NN)                                                                                        \
    case NN: hipExtLaunchKernelGGL((k_row_fwd<R, NN, V, MULTI>), dim3(blocks), dim3(RowCfg<R, NN, V>::T), 0, \
                                   st, e.a, e.b, 0, a, js, it); break;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
}
template <typename R, bool MULTI>
void launch_row_fwd_t(int n, int v, int blocks, hipStream_t st, StageEv e, const RowFwdArgs<R>& a,
                      Jobs<RowFwdArgs<R>> js, int it) {
    if constexpr (row_vars<R>() > 3) {
        if (v == 3) return launch_row_fwd_v<R, 3, MULTI>(n, blocks, st, e, a, js, it);
    }
    if (v == 2) launch_row_fwd_v<R, 2, MULTI>(n, blocks, st, e, a, js, it);
    else if (v == 1) launch_row_fwd_v<R, 1, MULTI>(n, blocks, st, e, a, js, it);
    else launch_row_fwd_v<R, 0, MULTI>(n, blocks, st, e, a, js, it);
}
template <typename R, int MODE, bool ZPASS, bool MULTI>
void launch_col_t(int n, int blocks, hipStream_t st, StageEv e, const ColArgs<R>& a, Jobs<ColArgs<R>> js,
                  int it) {
    switch (n) {
#define IBDL_C(NN)                                                                                        \
    case NN: {                                                                                            \
        constexpr int K = ZPASS ? ZRows<R, NN>::value : 1;                                                \
        static_assert(!ZPASS || K > 1, "K == 1 marks the 2-D column pass");                                \
        hipExtLaunchKernelGGL((k_col<R, NN, MODE, K, MULTI>), dim3(blocks), dim3(ColK<R, NN, K>::T), 0,       \
                              st, e.a, e.b, 0, a, js, it);                                                \
    } break;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
}
template <typename R, int OUT, int V, bool MULTI>
void launch_row_inv_v(int n, int blocks, hipStream_t st, StageEv e, const RowInvArgs<R>& a,
                      Jobs<RowInvArgs<R>> js, int it) {
    switch (n) {
#define IBDL_C(NN)                                                                                         \
    case NN: hipExtLaunchKernelGGL((k_row_inv<R, NN, OUT, V, MULTI>), dim3(blocks), dim3(RowCfg<R, NN, V>::T), \
                                   0, st, e.a, e.b, 0, a, js, it); break;
        IBDL_SIZES(IBDL_C)
#undef IBDL_C
    }
}
template <typename R, int OUT, bool MULTI>
void launch_row_inv_t(int n, int v, int blocks, hipStream_t st, StageEv e, const RowInvArgs<R>& a,
                      Jobs<RowInvArgs<R>> js, int it) {
    if constexpr (row_vars<R>() > 3) {
        if (v == 3) return launch_row_inv_v<R, OUT, 3, MULTI>(n, blocks, st, e, a, js, it);
    }
    if (v == 2) launch_row_inv_v<R, OUT, 2, MULTI>(n, blocks, st, e, a, js, it);
    else if (v == 1) launch_row_inv_v<R, OUT, 1, MULTI>(n, blocks, st, e, a, js, it);
    else launch_row_inv_v<R, OUT, 0, MULTI>(n, blocks, st, e, a, js, it);
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

// One pass of L^-1 for one or more jobs of the same dimension, grid size and
// precision: per stage a table of per-job arguments.

template <typename R>
struct PreparedT : PreparedPass {
    int n = 0, dim = 2;
    int out_mode = 0;  // 0: point output, 1: grid output, 2: both
    int min_nrhs = 1, total_rhs = 1, njobs = 1;
    int grid_in = 0;  // some job reads a forcing grid: its forward rows cover every line
    ibdl_plan tplan = nullptr;  // plan whose stage timing records this pass
    StageTable<RowFwdArgs<R>> rf[kRowVars];  // one table per row-block variant
    StageTable<ColArgs<R>> col[3];
    StageTable<RowInvArgs<R>> ri[kRowVars];
    StageTable<FinishArgs> fi;
    StageTable<PackArgs<R>> pk;  // strengths of the pass, packed before the forward rows

    void upload(Arena& ar, hipStream_t st) override {
        pk.upload(ar, st);
        for (auto& t : rf) t.upload(ar, st);
        for (auto& c : col) c.upload(ar, st);
        for (auto& t : ri) t.upload(ar, st);
        fi.upload(ar, st);
    }
    TuneKey key(int stage) const {
        return TuneKey{(int)sizeof(R), dim, n, stage, out_mode, tune_bucket(min_nrhs),
                       tune_bucket(total_rhs), njobs > 1 ? 1 : 0, stage == 0 ? grid_in : 0};
    }
    void fwd(int v, int it, hipStream_t st, StageEv e) {
        const auto& t = rf[v];
        go(t, [&](bool m) {
            if (m) launch_row_fwd_t<R, true>(n, v, t.blocks(), st, e, t.args[0], t.jobs(itp_), it);
            else launch_row_fwd_t<R, false>(n, v, t.blocks(), st, e, t.args[0], t.jobs(itp_), it);
        });
    }
    void inv(int v, int it, hipStream_t st, StageEv e) {
        const auto& t = ri[v];
        go(t, [&](bool m) {
            if (out_mode == 2) {
                if (m) launch_row_inv_t<R, 2, true>(n, v, t.blocks(), st, e, t.args[0], t.jobs(itp_), it);
                else launch_row_inv_t<R, 2, false>(n, v, t.blocks(), st, e, t.args[0], t.jobs(itp_), it);
            } else if (out_mode == 1) {
                if (m) launch_row_inv_t<R, 1, true>(n, v, t.blocks(), st, e, t.args[0], t.jobs(itp_), it);
                else launch_row_inv_t<R, 1, false>(n, v, t.blocks(), st, e, t.args[0], t.jobs(itp_), it);
            } else {
                if (m) launch_row_inv_t<R, 0, true>(n, v, t.blocks(), st, e, t.args[0], t.jobs(itp_), it);
                else launch_row_inv_t<R, 0, false>(n, v, t.blocks(), st, e, t.args[0], t.jobs(itp_), it);
            }
        });
    }
    // The row-block variant of a stage: the tuned choice for this pass's key; with no
    // choice yet, every variant runs (each produces the same output, since the
    // arithmetic of a line and of a point does not depend on the grouping), is timed
    // on its second run, and the fastest is kept.
    template <class F>
    int pick(int stage, int it, hipStream_t st, F&& launch) {
        const int f = tune_forced();
        if (f >= 0) return f < row_vars<R>() ? f : 0;
        int v = tune_lookup(key(stage));
        if (v >= 0) return v;
        if (!tune_enabled() || capturing()) return heuristic();
        // every shape once untimed, then kTuneRounds timed rounds over all shapes in
        // turn; a shape's time is its fastest run (a single sample per shape picked
        // a 20% slower 3-D spread shape in some processes)
        constexpr int kTuneRounds = 3;
        float ms_min[kRowVars];
        for (int c = 0; c < row_vars<R>(); ++c) {
            ms_min[c] = 1e30f;
            launch(c, StageEv{});
        }
        hipEvent_t e0, e1;
        IBDL_HIP_TRY(hipEventCreate(&e0));
        IBDL_HIP_TRY(hipEventCreate(&e1));
        for (int round = 0; round < kTuneRounds; ++round)
            for (int c = 0; c < row_vars<R>(); ++c) {
                launch(c, StageEv{e0, e1});
                IBDL_HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                IBDL_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                ms_min[c] = std::min(ms_min[c], ms);
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        float best = 1e30f;
        int bv = heuristic();
        for (int c = 0; c < row_vars<R>(); ++c)
            if (ms_min[c] < best) {
                best = ms_min[c];
                bv = c;
            }
        tune_store(key(stage), bv, best);
        return -1 - bv;  // already run
    }
    int heuristic() const { return min_nrhs >= 4 ? 2 : min_nrhs >= 2 ? 1 : 0; }
    template <class T, class F>
    static void go(const StageTable<T>& tb, F&& f) {
        if (tb.blocks() == 0) return;
        f(tb.multi());
    }
    void run(int it, hipStream_t st) override {
        int stage = 0;
        go(pk, [&](bool m) {
            const StageEv e = stage_events(tplan, stage++, "pack");
            if (m)
                hipExtLaunchKernelGGL((k_pack<R, true>), dim3(pk.blocks()), dim3(256), 0, st, e.a, e.b, 0, pk.args[0],
                                      pk.jobs(itp_), it);
            else
                hipExtLaunchKernelGGL((k_pack<R, false>), dim3(pk.blocks()), dim3(256), 0, st, e.a, e.b, 0,
                                      pk.args[0], pk.jobs(itp_), it);
        });
        {
            const int v = pick(0, it, st, [&](int c, StageEv e) { fwd(c, it, st, e); });
            const StageEv e = stage_events(tplan, stage++, "spread+fft_x");
            // a stage tuned just now has run already; with timing on it runs once
            // more (it overwrites its outputs from unchanged inputs) so that the
            // stage's events are recorded
            if (v >= 0) fwd(v, it, st, e);
            else if (e.a) fwd(-1 - v, it, st, e);
        }
        if (dim == 2) {
            const StageEv e = stage_events(tplan, stage++, "fft_y+symbol");
            go(col[0], [&](bool m) {
                if (m) launch_col_t<R, 1, false, true>(n, col[0].blocks(), st, e, col[0].args[0], col[0].jobs(itp_), it);
                else launch_col_t<R, 1, false, false>(n, col[0].blocks(), st, e, col[0].args[0], col[0].jobs(itp_), it);
            });
        } else {
            StageEv e = stage_events(tplan, stage++, "fft_y");
            go(col[0], [&](bool m) {
                if (m) launch_col_t<R, 0, false, true>(n, col[0].blocks(), st, e, col[0].args[0], col[0].jobs(itp_), it);
                else launch_col_t<R, 0, false, false>(n, col[0].blocks(), st, e, col[0].args[0], col[0].jobs(itp_), it);
            });
            e = stage_events(tplan, stage++, "fft_z+symbol");
            go(col[1], [&](bool m) {
                if (m) launch_col_t<R, 1, true, true>(n, col[1].blocks(), st, e, col[1].args[0], col[1].jobs(itp_), it);
                else launch_col_t<R, 1, true, false>(n, col[1].blocks(), st, e, col[1].args[0], col[1].jobs(itp_), it);
            });
            e = stage_events(tplan, stage++, "ifft_y");
            go(col[2], [&](bool m) {
                if (m) launch_col_t<R, 2, false, true>(n, col[2].blocks(), st, e, col[2].args[0], col[2].jobs(itp_), it);
                else launch_col_t<R, 2, false, false>(n, col[2].blocks(), st, e, col[2].args[0], col[2].jobs(itp_), it);
            });
        }
        {
            const int v = pick(1, it, st, [&](int c, StageEv e) { inv(c, it, st, e); });
            const StageEv e = stage_events(tplan, stage++, out_mode == 1 ? "ifft_x" : "ifft_x+interp");
            if (v >= 0) inv(v, it, st, e);
            else if (e.a) inv(-1 - v, it, st, e);
        }
        if (out_mode != 1) {
            StageEv e;
            e = stage_events(tplan, stage++, "finish");
            go(fi, [&](bool m) {
                if (m)
                    hipExtLaunchKernelGGL((k_finish<R, true>), dim3(fi.blocks()), dim3(FIN_T), 0, st, e.a, e.b, 0,
                                          fi.args[0], fi.jobs(itp_), it);
                else
                    hipExtLaunchKernelGGL((k_finish<R, false>), dim3(fi.blocks()), dim3(FIN_T), 0, st, e.a, e.b,
                                          0, fi.args[0], fi.jobs(itp_), it);
            });
        }
        IBDL_HIP_TRY(hipGetLastError());
    }
};

template <typename R>
std::unique_ptr<PreparedPass> prepare_t(const std::vector<PassJob>& jobs) {
    using PP = PlanPrec<R>;
    auto P = std::make_unique<PreparedT<R>>();
    const ibdl_plan p0 = jobs[0].p;
    const int n = p0->n;
    P->n = n;
    P->dim = p0->dim;
    P->out_mode = jobs[0].out.u ? (jobs[0].out.out ? 2 : 1) : 0;
    P->tplan = p0;
    int minr = 1 << 30, tot = 0;
    for (const PassJob& jb : jobs) {
        minr = std::min(minr, jb.nrhs);
        tot += jb.nrhs;
    }
    P->min_nrhs = minr;
    P->total_rhs = tot;
    P->njobs = (int)jobs.size();
    for (const PassJob& jb : jobs) P->grid_in |= jb.in.grid != nullptr;
    const int C = col_width<R>(n);
    const int NT = col_tiles<R>(n);
    const size_t plane = (size_t)NT * n * C;
    const int KZ = z_rows<R>(n);
    for (const PassJob& jb : jobs) {
        const ibdl_plan p = jb.p;
        const PipeIn& in = jb.in;
        const PipeOut& out = jb.out;
        const int nrhs = jb.nrhs;
        const bool dense_in = in.grid != nullptr;
        const bool dense_out = out.u != nullptr;
        cplx<R>* spec = reinterpret_cast<cplx<R>*>(p->ws.spec);
        const size_t sstride = p->spec_elems;

        // ---- row_fwd
        RowFwdArgs<R> ra{};
        ra.skip = in.skip;
        ra.lines = dense_in ? nullptr : p->spread_lines;
        ra.nproc = dense_in ? p->nlines : p->n_spread_lines;
        ra.M = p->M;
        auto view = [&](const Csr& c, const double* q, double coef) {
            CsrView<R> v{};
            v.q_stride = in.q_stride ? in.q_stride : (size_t)p->M;
            v.q_jstride = in.q_jstride;
            v.line_act = c.line_act;
            v.act_ptr = c.act_ptr;
            v.act_node = c.act_node;
            v.k = c.k;
            v.s = c.s;
            v.w = PP::w(c);
            v.nnz = (uint32_t)c.nnz;
            v.q = q;
            v.coef = coef;
            v.M = p->M;
            return v;
        };
        ra.dip = view(p->dip, in.q_dip, in.c_dip);
        // packing costs a launch per pass: it pays where a block serves several
        // right-hand sides of a large spread.  Measured, FP32: sphere 256^3 at 32 rhs
        // spread 0.75 -> 0.37 ms per apply, star 1024^2 at 32 rhs 45 -> 37 us (the
        // pack 4 us); at 1 rhs and in the batch of small instances the extra launch
        // made solves 2-4% slower.  FP64 (32-byte segments): sphere 256^3 spread
        // 1.03 -> 0.91 ms, star 1024^2 no gain (68.7 -> 67 us against a 4 us pack).
        constexpr int64_t kPackMinWork = sizeof(R) == 4 ? (int64_t)1 << 21 : (int64_t)1 << 24;  // entries x rhs
        // ws.qf is FP64-sized, so a mixed plan's FP64 passes pack too
        if (in.pack_q && in.q_dip && nrhs >= 4 && p->dip.nnz * (int64_t)nrhs >= kPackMinWork) {
            if (!p->ws.qf) throw Error{IBDL_ERR_HIP, "packed strengths requested without their workspace"};
            PackArgs<R> pa{};
            pa.q = in.q_dip;
            pa.q_stride = ra.dip.q_stride;
            pa.q_jstride = in.q_jstride;
            pa.M = p->M;
            pa.nrhs = nrhs;
            pa.nkb = (p->M + 255) / 256;
            pa.perm = p->perm;
            pa.qf = reinterpret_cast<R*>(p->ws.qf);
            P->pk.add(pa, pa.nkb * ((nrhs + 3) / 4));
            ra.dip.qf = pa.qf;
        }
        ra.mono = view(p->mono, in.q_mono, in.c_mono);
        ra.grid = in.grid;
        ra.cg = in.c_grid;
        ra.grid_stride = (size_t)p->nlines * n;
        ra.spec = spec;
        ra.spec_stride = sstride;
        ra.P = p->P;
        ra.tw = PP::tw(p);
        ra.nrhs = nrhs;
        // grid forcing: the row pass flags the lines it writes, per right-hand side;
        // the 3-D y pass then flags the planes it writes
        uint8_t* const lnz = dense_in ? p->ws.dmask : nullptr;
        uint8_t* const pnz = dense_in ? p->ws.dmask + (size_t)p->ws.cap_rhs * p->nlines : nullptr;
        if (dense_in && !p->ws.dmask) throw Error{IBDL_ERR_HIP, "grid-forcing pass without its line masks"};
        ra.lnz = lnz;
        ra.lnz_rhs = (size_t)p->nlines;
        for (int v = 0; v < kRowVars; ++v) {
            const int G = row_lines_per_block<R>(n, v);
            ra.nblk = (ra.nproc + G - 1) / G;
            P->rf[v].add(ra, ra.nblk * ((nrhs + kRowVarRB[v] - 1) / kRowVarRB[v]));
        }

        // ---- columns
        ColArgs<R> ca{};
        ca.skip = in.skip;
        ca.spec = spec;
        ca.rhs_stride = sstride;
        ca.width = p->W;
        ca.tw = PP::tw(p);
        ca.s2 = PP::s2(p);
        if (in.alpha_zero && sizeof(R) == 4 && p->dim == 2)
            throw Error{IBDL_ERR_HIP, "a mean-zero pass needs the FP64 pipeline"};
        ca.alpha = in.alpha_zero ? R(0) : (R)p->alpha;
        ca.norm = (R)(2.0 / ((double)p->nlines * (double)n));
        if constexpr (sizeof(R) == 4) {
            if (p->dim == 2 && !p->sym32) throw Error{IBDL_ERR_HIP, "2-D plan without its FP32 symbol table"};
            ca.sym = p->dim == 2 ? p->sym32 : nullptr;
        }
        ca.tile_stride = (size_t)n * C;
        ca.nrhs = nrhs;
        if (p->dim == 2) {
            ca.outer_list = nullptr;
            ca.outer_stride = 0;
            ca.es = C;
            ca.lmask = dense_in ? lnz : p->spread_line_mask;
            ca.lm_outer = 0; ca.lm_stride = 1;
            ca.lm_rhs = dense_in ? (size_t)p->nlines : 0;
            ca.smask = dense_out ? nullptr : p->gather_line_mask;
            ca.sm_outer = 0; ca.sm_stride = 1;
            ca.nouter = 1;
            P->col[0].add(ca, NT * nrhs);
        } else {
            ColArgs<R> y1 = ca;  // y forward over planes that hold forcing
            y1.outer_list = dense_in ? nullptr : p->spread_planes;
            y1.outer_stride = plane;
            y1.es = C;
            y1.lmask = dense_in ? lnz : p->spread_line_mask;
            y1.lm_outer = n; y1.lm_stride = 1;
            y1.lm_rhs = dense_in ? (size_t)p->nlines : 0;
            y1.onz = pnz;
            y1.onz_rhs = (size_t)n;
            y1.smask = nullptr;
            y1.nouter = dense_in ? n : p->n_spread_planes;
            P->col[0].add(y1, NT * y1.nouter * nrhs);
            ColArgs<R> z = ca;   // z forward, symbol, z inverse: blocks of KZ y-rows of one tile
            z.outer_list = nullptr;
            z.outer_stride = (size_t)KZ * C;
            z.es = plane;
            z.lmask = dense_in ? pnz : p->spread_plane_mask;
            z.lm_outer = 0; z.lm_stride = 1;
            z.lm_rhs = dense_in ? (size_t)n : 0;
            z.smask = dense_out ? nullptr : p->gather_plane_mask;
            z.sm_outer = 0; z.sm_stride = 1;
            z.nouter = n / KZ;
            P->col[1].add(z, NT * z.nouter * nrhs);
            ColArgs<R> y2 = ca;  // y inverse over planes something is read from
            y2.outer_list = dense_out ? nullptr : p->gather_planes;
            y2.outer_stride = plane;
            y2.es = C;
            y2.lmask = nullptr;
            y2.smask = dense_out ? nullptr : p->gather_line_mask;
            y2.sm_outer = n; y2.sm_stride = 1;
            y2.nouter = dense_out ? n : p->n_gather_planes;
            P->col[2].add(y2, NT * y2.nouter * nrhs);
        }

        // ---- row_inv
        RowInvArgs<R> ia{};
        ia.skip = in.skip;
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
        ia.nrhs = nrhs;
        for (int v = 0; v < kRowVars; ++v) {
            const int G = row_lines_per_block<R>(n, v);
            ia.nblk = (ia.nproc + G - 1) / G;
            P->ri[v].add(ia, ia.nblk * ((nrhs + kRowVarRB[v] - 1) / kRowVarRB[v]));
        }

        // ---- finish
        if (out.out) {
            FinishArgs fa{};
            fa.skip = in.skip;
            fa.perm = p->perm;
            fa.M = p->M;
            fa.gpp = p->gpp;
            fa.nblk = (p->M + FIN_T - 1) / FIN_T;
            fa.part = p->ws.part;
            fa.part_stride = ia.part_stride;
            fa.out = out.out;
            fa.out_stride = out.out_stride ? out.out_stride : (size_t)p->M;
            fa.out_jstride = out.out_jstride;
            fa.cA = out.cA;
            fa.in = out.in;
            fa.in_stride = out.in_stride ? out.in_stride : (size_t)p->M;
            fa.in_jstride = out.in_jstride;
            fa.cB = out.cB;
            fa.in2 = out.in2;
            fa.in2_stride = out.in2_stride ? out.in2_stride : (size_t)p->M;
            fa.cC = out.cC;
            fa.V = out.dots_V;
            fa.vstride_rhs = out.dots_vstride;
            fa.nv = out.dots_nv;
            fa.dots = out.dots;
            fa.dots_rhs = out.dots_rhs;
            fa.dstride = out.dots_stride;
            P->fi.add(fa, fa.nblk * nrhs);
        }
    }
    return P;
}

}  // namespace ibdl
