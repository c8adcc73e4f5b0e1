// Unpreconditioned restarted GMRES on the boundary density (Sec. 5.3), FP64 on
// the device for every right-hand side at once.
//
// Arnoldi step j of right-hand side r:  w = A v_j (one pass of the operator),
// h_ij = <w, v_i> and w -= sum_i h_ij v_i done twice (classical Gram-Schmidt
// applied twice), h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}; the previous Givens
// rotations are applied to column j, a new rotation zeroes h_{j+1,j}, and the
// rotated right-hand side g gives the residual estimate |g_{j+1}|.  All inner
// products are two-level block reductions in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "plan.h"

namespace ibdl {

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

constexpr int GT = 256;             // threads per block
constexpr int GPER = 1;             // elements per thread
constexpr int GCHUNK = GT * GPER;   // elements per block
constexpr int FIN_BLOCK = 256;      // points per block of the operator's finishing kernel

enum { ST_DONE = 0, ST_ITERS = 1, ST_STATUS = 2, ST_J = 3 };

__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < GT / 64; ++i) t += sh[i];
    return t;  // valid in thread 0
}

// Block sums of nv per-thread values at once: each wave reduces its values with
// cross-lane shuffles, one LDS write per wave and value, one barrier, then
// thread i adds the wave totals of value i (fixed order).  out[i] valid in
// threads i < nv after the call; sh holds GT/64 * nv doubles.
template <int MAXV>
__device__ __forceinline__ void block_multi_sum(double (&v)[MAXV], int nv, double* sh, double* out) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        if (i < nv) {
            double t = v[i];
            for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
            if (l == 0) sh[w * MAXV + i] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        double t = 0.0;
        for (int ww = 0; ww < GT / 64; ++ww) t += sh[ww * MAXV + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

struct KArgs {
    double* V;          // [rhs][m+1][M]
    size_t vstride;
    int M, m, nblk;
    int nblk_dots;      // blocks of the operator's fused first inner products
    double* part;       // [rhs][blocks][m+2] (two banks: part and part2)
    double* part2;
    size_t pstride;     // per rhs
    double* hcol;       // [rhs][m+2]
    double* H;          // [rhs][m][m+1] column j at H + j*(m+1)
    double* cs;         // [rhs][m]
    double* sn;
    double* g;          // [rhs][m+1]
    double* y;          // [rhs][m]
    double* bnorm;      // [rhs]
    double* resid;      // [rhs]
    int32_t* state;     // [rhs][4]
    const double* tolv; // [rhs] tolerance relative to ||b_r||
};

// sum of squares of x over each block's chunk
__global__ __launch_bounds__(GT) void k_sumsq(const double* __restrict__ x, size_t xstride, int M,
                                              double* part, size_t pstride) {
    __shared__ double sh[GT / 64];
    const int rhs = blockIdx.y;
    const double* xr = x + (size_t)rhs * xstride;
    double acc = 0.0;
    for (int i = 0; i < GPER; ++i) {
        const size_t m = (size_t)blockIdx.x * GCHUNK + i * GT + threadIdx.x;
        if (m < (size_t)M) acc += xr[m] * xr[m];
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(size_t)rhs * pstride + blockIdx.x] = t;
}

__global__ void k_set_bnorm(const double* __restrict__ part, size_t pstride, int nblk,
                            double* bnorm, int32_t* state, const int32_t* skip, int nrhs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)r * pstride + b];
    bnorm[r] = sqrt(s);
    state[4 * r + ST_DONE] = skip[r];
    state[4 * r + ST_ITERS] = 0;
    state[4 * r + ST_STATUS] = isfinite(s) ? IBDL_OK : IBDL_ERR_NUMERIC;
    state[4 * r + ST_J] = 0;
}

// start a cycle: v_0 = r / ||r||, g = (||r||, 0, ...); rhs already done are left alone
__global__ __launch_bounds__(GT) void k_init_cycle(const double* __restrict__ rv, size_t rstride,
                                                   KArgs a) {
    const int rhs = blockIdx.y;
    int32_t* st = a.state + 4 * rhs;
    if (st[ST_DONE]) return;
    double s = 0.0;
    for (int b = 0; b < a.nblk; ++b) s += a.part[(size_t)rhs * a.pstride + b];
    const double beta = sqrt(s);
    const double bn = a.bnorm[rhs];
    const bool done = !(bn > 0.0) || beta <= a.tolv[rhs] * bn || !(beta > 0.0);
    const double inv = (beta > 0.0) ? 1.0 / beta : 0.0;
    double* v0 = a.V + (size_t)rhs * a.vstride;
    const double* r = rv + (size_t)rhs * rstride;
    for (int i = 0; i < GPER; ++i) {
        const size_t m = (size_t)blockIdx.x * GCHUNK + i * GT + threadIdx.x;
        if (m < (size_t)a.M) v0[m] = r[m] * inv;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double* g = a.g + (size_t)rhs * (a.m + 1);
        g[0] = beta;
        for (int i = 1; i <= a.m; ++i) g[i] = 0.0;
        a.resid[rhs] = bn > 0.0 ? beta / bn : 0.0;
        st[ST_J] = 0;
        if (!isfinite(s)) st[ST_STATUS] = IBDL_ERR_NUMERIC;
        if (done || !isfinite(s)) st[ST_DONE] = 1;
    }
}

// h = sum of the block partials of pass `pass`; w -= V h; then the partials of
// the next quantity: pass 0 -> <w, v_i> again, pass 1 -> ||w||^2
__global__ __launch_bounds__(GT) void k_orth(KArgs a, int j, int pass) {
    __shared__ double sh[GT / 64];
    __shared__ double hs[256];
    const int rhs = blockIdx.y;
    if (a.state[4 * rhs + ST_DONE]) return;
    const double* pin = (pass == 0 ? a.part : a.part2) + (size_t)rhs * a.pstride;
    double* pout = (pass == 0 ? a.part2 : a.part) + (size_t)rhs * a.pstride;
    const int nb_in = pass == 0 ? a.nblk_dots : a.nblk;
    for (int vi = threadIdx.x; vi <= j; vi += GT) {
        double s = 0.0;
        for (int b = 0; b < nb_in; ++b) s += pin[(size_t)b * (a.m + 2) + vi];
        hs[vi] = s;
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double* hc = a.hcol + (size_t)rhs * (a.m + 2);
        for (int vi = 0; vi <= j; ++vi) hc[vi] = (pass == 0 ? 0.0 : hc[vi]) + hs[vi];
    }
    double* V = a.V + (size_t)rhs * a.vstride;
    double* w = V + (size_t)(j + 1) * a.M;
    double wl[GPER];
    for (int i = 0; i < GPER; ++i) {
        const size_t m = (size_t)blockIdx.x * GCHUNK + i * GT + threadIdx.x;
        if (m < (size_t)a.M) {
            double acc = w[m];
            for (int vi = 0; vi <= j; ++vi) acc -= hs[vi] * V[(size_t)vi * a.M + m];
            wl[i] = acc;
            w[m] = acc;
        } else {
            wl[i] = 0.0;
        }
    }
    if (pass == 0) {
        // <w, v_i> for i <= j, 16 at a time
        __shared__ double msh[(GT / 64) * 16];
        __shared__ double mout[16];
        for (int v0 = 0; v0 <= j; v0 += 16) {
            const int nv = imin(16, j + 1 - v0);
            double acc[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = 0.0;
            for (int i = 0; i < GPER; ++i) {
                const size_t m = (size_t)blockIdx.x * GCHUNK + i * GT + threadIdx.x;
                if (m < (size_t)a.M) {
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                        if (u < nv) acc[u] += V[(size_t)(v0 + u) * a.M + m] * wl[i];
                }
            }
            block_multi_sum<16>(acc, nv, msh, mout);
            if (threadIdx.x < nv) pout[(size_t)blockIdx.x * (a.m + 2) + v0 + threadIdx.x] = mout[threadIdx.x];
        }
    } else {
        double acc = 0.0;
        for (int i = 0; i < GPER; ++i) acc += wl[i] * wl[i];
        const double t = block_sum(acc, sh);
        if (threadIdx.x == 0) pout[(size_t)blockIdx.x * (a.m + 2)] = t;
    }
}

// v_{j+1} = w / ||w||; block 0 applies the Givens rotations and updates the state
__global__ __launch_bounds__(GT) void k_normalize_givens(KArgs a, int j) {
    const int rhs = blockIdx.y;
    int32_t* st = a.state + 4 * rhs;
    if (st[ST_DONE]) return;
    const double* pin = a.part + (size_t)rhs * a.pstride;
    double s = 0.0;
    for (int b = 0; b < a.nblk; ++b) s += pin[(size_t)b * (a.m + 2)];
    const double hn = sqrt(s);
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    double* w = a.V + (size_t)rhs * a.vstride + (size_t)(j + 1) * a.M;
    for (int i = 0; i < GPER; ++i) {
        const size_t m = (size_t)blockIdx.x * GCHUNK + i * GT + threadIdx.x;
        if (m < (size_t)a.M) w[m] *= inv;
    }
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const double* hc = a.hcol + (size_t)rhs * (a.m + 2);
    double* Hj = a.H + (size_t)rhs * a.m * (a.m + 1) + (size_t)j * (a.m + 1);
    double* cs = a.cs + (size_t)rhs * a.m;
    double* sn = a.sn + (size_t)rhs * a.m;
    double* g = a.g + (size_t)rhs * (a.m + 1);
    for (int i = 0; i <= j; ++i) Hj[i] = hc[i];
    Hj[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = t;
    }
    const double den = hypot(Hj[j], Hj[j + 1]);
    const double c = den > 0.0 ? Hj[j] / den : 1.0;
    const double sv = den > 0.0 ? Hj[j + 1] / den : 0.0;
    cs[j] = c;
    sn[j] = sv;
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    g[j + 1] = -sv * g[j];
    g[j] = c * g[j];
    const double res = fabs(g[j + 1]) / a.bnorm[rhs];
    a.resid[rhs] = res;
    st[ST_ITERS] += 1;
    st[ST_J] = j + 1;
    if (!isfinite(res) || !isfinite(s)) {
        st[ST_STATUS] = IBDL_ERR_NUMERIC;
        st[ST_DONE] = 1;
    } else if (res <= a.tolv[rhs] || !(hn > 0.0)) {
        st[ST_DONE] = 1;
    }
}

// y = R^-1 g over the steps of the current cycle, then mark the cycle as consumed
__global__ void k_backsolve(KArgs a, int nrhs) {
    const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
    if (rhs >= nrhs) return;
    const int jr = a.state[4 * rhs + ST_J];
    const double* H = a.H + (size_t)rhs * a.m * (a.m + 1);
    const double* g = a.g + (size_t)rhs * (a.m + 1);
    double* y = a.y + (size_t)rhs * a.m;
    for (int i = jr - 1; i >= 0; --i) {
        double t = g[i];
        for (int k = i + 1; k < jr; ++k) t -= H[(size_t)k * (a.m + 1) + i] * y[k];
        const double d = H[(size_t)i * (a.m + 1) + i];
        y[i] = d != 0.0 ? t / d : 0.0;
    }
}

// x += V[0..jr) y ; then the cycle position is reset
__global__ __launch_bounds__(GT) void k_update_x(KArgs a, double* x, size_t xstride) {
    const int rhs = blockIdx.y;
    const int jr = a.state[4 * rhs + ST_J];
    if (jr == 0) return;
    const double* V = a.V + (size_t)rhs * a.vstride;
    const double* y = a.y + (size_t)rhs * a.m;
    double* xr = x + (size_t)rhs * xstride;
    for (int i = 0; i < GPER; ++i) {
        const size_t m = (size_t)blockIdx.x * GCHUNK + i * GT + threadIdx.x;
        if (m < (size_t)a.M) {
            double acc = xr[m];
            for (int vi = 0; vi < jr; ++vi) acc += y[vi] * V[(size_t)vi * a.M + m];
            xr[m] = acc;
        }
    }
}

__global__ void k_reset_j(int32_t* state, int nrhs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrhs) state[4 * r + ST_J] = 0;
}

__global__ void k_fill0_masked(double* x, size_t stride, int M, const int32_t* skip) {
    const int rhs = blockIdx.y;
    if (skip[rhs]) return;
    for (int i = 0; i < GPER; ++i) {
        const size_t mm = (size_t)blockIdx.x * GCHUNK + i * GT + threadIdx.x;
        if (mm < (size_t)M) x[(size_t)rhs * stride + mm] = 0.0;
    }
}

__global__ void k_copy(double* dst, const double* src, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------------ host
static void ensure_krylov(ibdl_plan p, int nrhs, int m) {
    Krylov& k = p->kr;
    if (k.cap_rhs >= nrhs && k.cap_m >= m) return;
    const int M = p->M;
    const int nblk = (M + GCHUNK - 1) / GCHUNK;
    const int nbmax = std::max(nblk, (M + FIN_BLOCK - 1) / FIN_BLOCK);
    nrhs = std::max(nrhs, k.cap_rhs);
    m = std::max(m, k.cap_m);
    auto A = [&](size_t n) { return reinterpret_cast<double*>(dev_alloc(p, n * sizeof(double))); };
    k.V = A((size_t)nrhs * (m + 1) * M);
    k.H = A((size_t)nrhs * m * (m + 1));
    k.cs = A((size_t)nrhs * m);
    k.sn = A((size_t)nrhs * m);
    k.g = A((size_t)nrhs * (m + 1));
    k.y = A((size_t)nrhs * m);
    k.partial = A((size_t)nrhs * nbmax * (m + 2) * 2);
    k.hcol = A((size_t)nrhs * (m + 2));
    k.bnorm = A(nrhs);
    k.resid = A(nrhs);
    k.tolv = A(nrhs);
    k.b = A((size_t)nrhs * M);
    k.r = A((size_t)nrhs * M);
    k.rr = A((size_t)nrhs * M);
    k.d = A((size_t)nrhs * M);
    k.state = reinterpret_cast<int32_t*>(dev_alloc(p, (size_t)nrhs * 4 * sizeof(int32_t)));
    k.skip = reinterpret_cast<int32_t*>(dev_alloc(p, (size_t)nrhs * sizeof(int32_t)));
    if (k.host_pinned) (void)hipHostFree(k.host_pinned);
    k.host_pinned = nullptr;
    IBDL_HIP_TRY(hipHostMalloc(&k.host_pinned, (size_t)nrhs * 64 + 64));
    k.cap_rhs = nrhs;
    k.cap_m = m;
    k.nblk = nblk;
}

void apply_operator(ibdl_plan p, int nrhs, const double* q, size_t qstride, double* out,
                    size_t ostride, hipStream_t st);

// r = b - A x for every rhs (operator in FP64 when fp64, else the plan's precision)
static void residual(ibdl_plan p, int nrhs, const double* b, const double* x, double* r,
                     hipStream_t st, bool fp64) {
    // A x = -S* L^-1 S~ x + s x/2, so b - A x = S* L^-1 S~ x - s x/2 + b
    PipeIn in;
    in.q_dip = x;
    in.c_dip = 1.0;
    PipeOut out;
    out.out = r;
    out.cA = 1.0;
    out.in = x;
    out.cB = p->bc == IBDL_DIRICHLET ? -0.5 : 0.5;
    out.in2 = b;
    out.cC = 1.0;
    run_pipeline(p, nrhs, in, out, st, fp64);
}

// host copies of per-rhs norms: sqrt of the summed block partials of k_sumsq
static void norms(ibdl_plan p, int nrhs, const double* x, hipStream_t st, std::vector<double>& out) {
    Krylov& k = p->kr;
    const size_t pstride = (size_t)k.nblk;
    hipLaunchKernelGGL(k_sumsq, dim3(k.nblk, nrhs), dim3(GT), 0, st, x, (size_t)p->M, p->M, k.partial,
                       pstride);
    std::vector<double> hp((size_t)nrhs * pstride);
    IBDL_HIP_TRY(hipMemcpyAsync(hp.data(), k.partial, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    IBDL_HIP_TRY(hipStreamSynchronize(st));
    out.assign(nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r) {
        double s = 0.0;
        for (int b = 0; b < k.nblk; ++b) s += hp[(size_t)r * pstride + b];
        out[r] = std::sqrt(s);
    }
}

struct KrylovResult {
    std::vector<int> iters, status;
    std::vector<double> est;
};

// Restarted GMRES on A x = b with the operator in the plan's precision, for every
// rhs not marked in skip.  x holds the initial iterate (x_zero: it is set to 0).
// tol[r] is relative to ||b_r||.  Iterations add to res.iters.
static void krylov(ibdl_plan p, int nrhs, const double* b, double* x, bool x_zero,
                   const std::vector<double>& tol, int m, int maxit, const std::vector<int>& skip,
                   hipStream_t st, KrylovResult& res) {
    const int M = p->M;
    Krylov& k = p->kr;
    const int nblk = k.nblk;
    KArgs a{};
    a.V = k.V;
    a.vstride = (size_t)(m + 1) * M;
    a.M = M;
    a.m = m;
    a.nblk = nblk;
    a.nblk_dots = (M + FIN_BLOCK - 1) / FIN_BLOCK;
    a.part = k.partial;
    a.pstride = (size_t)std::max(nblk, a.nblk_dots) * (m + 2);
    a.part2 = k.partial + (size_t)nrhs * a.pstride;
    a.hcol = k.hcol;
    a.H = k.H;
    a.cs = k.cs;
    a.sn = k.sn;
    a.g = k.g;
    a.y = k.y;
    a.bnorm = k.bnorm;
    a.resid = k.resid;
    a.state = k.state;
    a.tolv = k.tolv;
    const dim3 vg(nblk, nrhs);
    const size_t tot = (size_t)nrhs * M;

    // per-rhs tolerances and skip flags
    double* hbuf = reinterpret_cast<double*>(k.host_pinned);
    int32_t* hint = reinterpret_cast<int32_t*>(hbuf + nrhs);
    for (int r = 0; r < nrhs; ++r) {
        hbuf[r] = tol[r];
        hint[r] = skip[r];
    }
    IBDL_HIP_TRY(hipMemcpyAsync(k.tolv, hbuf, nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    IBDL_HIP_TRY(hipMemcpyAsync(k.skip, hint, nrhs * sizeof(int32_t), hipMemcpyHostToDevice, st));

    hipLaunchKernelGGL(k_sumsq, vg, dim3(GT), 0, st, b, (size_t)M, M, k.partial, a.pstride);
    hipLaunchKernelGGL(k_set_bnorm, dim3((nrhs + 63) / 64), dim3(64), 0, st, k.partial, a.pstride, nblk,
                       k.bnorm, k.state, k.skip, nrhs);
    const double* r0 = b;
    if (x_zero) {
        hipLaunchKernelGGL(k_fill0_masked, vg, dim3(GT), 0, st, x, (size_t)M, M, k.skip);
    } else {
        residual(p, nrhs, b, x, k.r, st, false);
        r0 = k.r;
    }
    hipLaunchKernelGGL(k_sumsq, vg, dim3(GT), 0, st, r0, (size_t)M, M, k.partial, a.pstride);
    hipLaunchKernelGGL(k_init_cycle, vg, dim3(GT), 0, st, r0, (size_t)M, a);

    int32_t* hstate = reinterpret_cast<int32_t*>(hbuf + 2 * nrhs);
    double* hres_p = hbuf + 4 * nrhs;
    auto all_done = [&]() {
        IBDL_HIP_TRY(hipMemcpyAsync(hstate, k.state, (size_t)nrhs * 4 * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, st));
        IBDL_HIP_TRY(hipMemcpyAsync(hres_p, k.resid, (size_t)nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
        IBDL_HIP_TRY(hipStreamSynchronize(st));
        for (int r = 0; r < nrhs; ++r)
            if (!hstate[4 * r + ST_DONE]) return false;
        return true;
    };
    // Arnoldi step j for every rhs still running (kernels skip finished ones)
    auto iteration = [&](int j) {
        PipeIn in;
        in.q_dip = k.V + (size_t)j * M;
        in.c_dip = 1.0;
        in.q_stride = a.vstride;
        in.skip = k.state;
        PipeOut o;
        o.out = k.V + (size_t)(j + 1) * M;
        o.out_stride = a.vstride;
        o.cA = -1.0;
        o.in = k.V + (size_t)j * M;
        o.in_stride = a.vstride;
        o.cB = p->bc == IBDL_DIRICHLET ? 0.5 : -0.5;
        o.dots_V = k.V;
        o.dots_vstride = a.vstride;
        o.dots_nv = j + 1;
        o.dots = a.part;
        o.dots_rhs = a.pstride;
        o.dots_stride = m + 2;
        run_pipeline(p, nrhs, in, o, st);
        hipLaunchKernelGGL(k_orth, vg, dim3(GT), 0, st, a, j, 0);
        hipLaunchKernelGGL(k_orth, vg, dim3(GT), 0, st, a, j, 1);
        hipLaunchKernelGGL(k_normalize_givens, vg, dim3(GT), 0, st, a, j);
    };
    // how many steps to queue before looking at the state again: the steps the
    // slowest rhs needs at its observed rate of residual reduction (1..8)
    auto next_chunk = [&](int done_steps, const std::vector<double>& prev) {
        int need = 3;
        if (done_steps > 0) {
            need = 1;
            for (int r = 0; r < nrhs; ++r) {
                if (hstate[4 * r + ST_DONE]) continue;
                const double now = hres_p[r], before = prev[r];
                int nr = 8;
                if (now > 0.0 && before > now) {
                    const double rate = std::pow(now / before, 1.0 / done_steps);
                    if (rate < 1.0) nr = (int)std::ceil(std::log(tol[r] / now) / std::log(rate));
                }
                need = std::max(need, std::min(std::max(nr, 1), 8));
            }
        }
        return need;
    };

    int total = 0;
    bool finished = all_done();
    while (!finished) {
        int j = 0;
        int last = 0;
        std::vector<double> prev(hres_p, hres_p + nrhs);
        bool stop = false;
        while (j < m) {
            const int chunk = std::min({next_chunk(last, prev), m - j, maxit - total});
            prev.assign(hres_p, hres_p + nrhs);
            for (int t = 0; t < chunk; ++t) iteration(j + t);
            j += chunk;
            total += chunk;
            last = chunk;
            if (all_done() || total >= maxit) {
                stop = true;
                break;
            }
        }
        hipLaunchKernelGGL(k_backsolve, dim3((nrhs + 63) / 64), dim3(64), 0, st, a, nrhs);
        hipLaunchKernelGGL(k_update_x, vg, dim3(GT), 0, st, a, x, (size_t)M);
        hipLaunchKernelGGL(k_reset_j, dim3((nrhs + 63) / 64), dim3(64), 0, st, k.state, nrhs);
        if (stop) break;
        // restart the rhs still running from their current iterate
        residual(p, nrhs, b, x, k.r, st, false);
        hipLaunchKernelGGL(k_sumsq, vg, dim3(GT), 0, st, k.r, (size_t)M, M, k.partial, a.pstride);
        hipLaunchKernelGGL(k_init_cycle, vg, dim3(GT), 0, st, k.r, (size_t)M, a);
        finished = all_done();
    }
    IBDL_HIP_TRY(hipGetLastError());
    std::vector<double> hres(nrhs);
    IBDL_HIP_TRY(hipMemcpyAsync(hres.data(), k.resid, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    IBDL_HIP_TRY(hipMemcpyAsync(hstate, k.state, (size_t)nrhs * 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    IBDL_HIP_TRY(hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) {
        if (skip[r]) continue;
        res.iters[r] += hstate[4 * r + ST_ITERS];
        res.est[r] = hres[r];
        int s = hstate[4 * r + ST_STATUS];
        if (s == IBDL_OK && !(hres[r] <= tol[r])) s = IBDL_ERR_NOCONV;
        res.status[r] = s;
    }
}

__global__ void k_axpy_masked(double* x, const double* d, size_t stride, int M, const int32_t* skip) {
    const int rhs = blockIdx.y;
    if (skip[rhs]) return;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (size_t)M) x[(size_t)rhs * stride + i] += d[(size_t)rhs * stride + i];
}

void gmres_solve(ibdl_plan p, int nrhs, const double* data, const double* g, const ibdl_solve_opts& o,
                 double* sol, ibdl_solve_info* info, hipStream_t st, int* overall) {
    const int M = p->M;
    const int m = o.restart;
    ensure_krylov(p, nrhs, m);
    Krylov& k = p->kr;
    const size_t tot = (size_t)nrhs * M;

    // right-hand side b in FP64 (Dirichlet: U_b - S* L^-1 g~; Neumann: S* L^-1 (S V_b - g~))
    {
        PipeIn in;
        PipeOut out;
        out.out = k.b;
        if (p->bc == IBDL_DIRICHLET) {
            if (g) {
                in.grid = g;
                in.c_grid = 1.0;
                out.cA = -1.0;
                out.in = data;
                out.cB = 1.0;
                run_pipeline(p, nrhs, in, out, st, true);
            } else {
                hipLaunchKernelGGL(k_copy, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, k.b, data, tot);
            }
        } else {
            in.q_mono = data;
            in.c_mono = 1.0;
            if (g) {
                in.grid = g;
                in.c_grid = -1.0;
            }
            out.cA = 1.0;
            run_pipeline(p, nrhs, in, out, st, true);
        }
    }
    std::vector<double> bn;
    norms(p, nrhs, k.b, st, bn);

    KrylovResult res;
    res.iters.assign(nrhs, 0);
    res.status.assign(nrhs, IBDL_OK);
    res.est.assign(nrhs, 0.0);
    std::vector<double> tol(nrhs, o.tol);
    std::vector<int> skip(nrhs, 0);
    std::vector<double> truer(nrhs, -1.0);
    std::vector<int> fp64_applies(nrhs, 0);

    if (o.x0) {
        hipLaunchKernelGGL(k_copy, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, sol, o.x0, tot);
    }
    krylov(p, nrhs, k.b, sol, o.x0 == nullptr, tol, m, o.maxit, skip, st, res);

    if (p->prec == IBDL_PREC_MIXED) {
        // FP64 iterative refinement: r = b - A x with the FP64 operator, correct
        // with the FP32-operator Krylov solve of A d = r, x += d.
        for (int round = 0; round < 5; ++round) {
            residual(p, nrhs, k.b, sol, k.rr, st, true);
            std::vector<double> rn;
            norms(p, nrhs, k.rr, st, rn);
            bool all = true;
            for (int r = 0; r < nrhs; ++r) {
                fp64_applies[r] += skip[r] ? 0 : 1;
                const double rel = bn[r] > 0.0 ? rn[r] / bn[r] : 0.0;
                if (!skip[r]) {
                    truer[r] = rel;
                    res.est[r] = rel;
                }
                if (!std::isfinite(rel)) {
                    res.status[r] = IBDL_ERR_NUMERIC;
                    skip[r] = 1;
                } else if (rel <= o.tol || res.status[r] == IBDL_ERR_NUMERIC) {
                    if (res.status[r] == IBDL_ERR_NOCONV) res.status[r] = IBDL_OK;
                    skip[r] = 1;
                } else {
                    all = false;
                    // reduce the correction's residual to the target, no further than the FP32 floor
                    tol[r] = std::max(o.tol * bn[r] / rn[r], 1e-6);
                }
            }
            if (all || round == 4) {
                for (int r = 0; r < nrhs; ++r)
                    if (!(truer[r] <= o.tol) && res.status[r] == IBDL_OK) res.status[r] = IBDL_ERR_NOCONV;
                break;
            }
            int used = 0;
            for (int r = 0; r < nrhs; ++r) used = std::max(used, res.iters[r]);
            const int left = o.maxit - used;
            if (left <= 0) {
                for (int r = 0; r < nrhs; ++r)
                    if (!skip[r]) res.status[r] = IBDL_ERR_NOCONV;
                break;
            }
            krylov(p, nrhs, k.rr, k.d, true, tol, m, left, skip, st, res);
            hipLaunchKernelGGL(k_axpy_masked, dim3((M + 255) / 256, nrhs), dim3(256), 0, st, sol, k.d,
                               (size_t)M, M, k.skip);
        }
    } else if (o.true_residual) {
        residual(p, nrhs, k.b, sol, k.rr, st, true);
        std::vector<double> rn;
        norms(p, nrhs, k.rr, st, rn);
        for (int r = 0; r < nrhs; ++r) {
            truer[r] = bn[r] > 0.0 ? rn[r] / bn[r] : 0.0;
            fp64_applies[r] = 1;
        }
    }
    IBDL_HIP_TRY(hipStreamSynchronize(st));

    int worst = IBDL_OK;
    for (int r = 0; r < nrhs; ++r) {
        const int s = res.status[r];
        if (info) {
            info[r].iters = res.iters[r];
            info[r].rel_resid_est = res.est[r];
            info[r].rel_resid_true = truer[r];
            info[r].status = s;
            info[r].fp64_applies = fp64_applies[r];
        }
        if (s == IBDL_ERR_NUMERIC) worst = IBDL_ERR_NUMERIC;
        else if (s == IBDL_ERR_NOCONV && worst == IBDL_OK) worst = IBDL_ERR_NOCONV;
    }
    *overall = worst;
}

}  // namespace ibdl
