// The completed IBDL formulation for the Poisson equation (Sec. 5.4.1, App. C).
//
// For alpha = 0 and Dirichlet data the completed system is, for z = [Q; ubar],
//     -S* D0^-1 (S~ + eta S) Q + Q/2 + ubar 1 = U_b - S* D0^-1 g~
//     eta sum_k w_k Q_k                         = h^d sum_x g~(x)
// with D0^-1 the mean-zero inverse of the periodic Laplacian, and the grid
// solution is u = D0^-1 (g~ - (S~ + eta S) Q) + ubar.  The operator applied to z
// (ibdl_apply) is the bordered matrix itself.  Solves eliminate the border: with
// K = Q/2 - S* D0^-1 (S~ + eta S) Q (the IBDL operator plus the single layer of
// the completion, invertible by the completion), K Q1 = U_b - S* D0^-1 g~ and
// K Q2 = 1 (once per plan), ubar = (eta w.Q1 - h^d sum g~) / (eta w.Q2) and
// Q = Q1 - ubar Q2 satisfy both rows; every K solve is the device GMRES of the
// other formulations with the single-layer term added to the operator pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "solve.h"

namespace ibdl {

namespace {

constexpr int RT = 256;

// one block per right-hand side: out[r * os] = coef * sum_k w[k] x[r * xs + k]
// (each thread its strided share, then a fixed-order tree)
__global__ __launch_bounds__(RT) void k_wsum(const double* __restrict__ x, size_t xs, const double* __restrict__ w,
                                            int M, double coef, double* out, size_t os) {
    __shared__ double sh[RT];
    const int r = blockIdx.x;
    double acc = 0.0;
    for (int k = threadIdx.x; k < M; k += RT) acc = fmac(w[k], x[(size_t)r * xs + k], acc);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = RT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)r * os] = coef * sh[0];
}

// grid sums in two fixed-order stages: block b of right-hand side r (blockIdx.y)
// sums its chunk into part[r * nb + b]; then one thread per rhs adds the parts
__global__ __launch_bounds__(RT) void k_gsum_part(const double* __restrict__ g, size_t len, int nb, double* part) {
    __shared__ double sh[RT];
    const int r = blockIdx.y;
    const size_t chunk = (len + nb - 1) / nb;
    const size_t b0 = (size_t)blockIdx.x * chunk, b1 = std::min(len, b0 + chunk);
    double acc = 0.0;
    for (size_t i = b0 + threadIdx.x; i < b1; i += RT) acc += g[(size_t)r * len + i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = RT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)r * nb + blockIdx.x] = sh[0];
}
__global__ void k_gsum_final(const double* __restrict__ part, int nb, int nrhs, double coef, double* out, size_t os) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)r * nb + b];
    out[(size_t)r * os] = coef * s;
}

// z[r][k] += z[r][M] for k < M (the ubar column of the bordered matrix), the
// border row z[r][M] = wq[r] already written; zin gives ubar
__global__ void k_add_last(const double* __restrict__ zin, size_t is, double* z, size_t os, int M) {
    const int r = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    z[(size_t)r * os + k] += zin[(size_t)r * is + M];
}

// sol[r] = [Q1 - ubar Q2; ubar], ubar = (c1[r] - b2[r]) / c2 (c1 = eta w.Q1, c2 = eta w.Q2)
__global__ void k_combine(const double* __restrict__ q1, const double* __restrict__ q2, const double* __restrict__ c1,
                          const double* __restrict__ b2, const double* __restrict__ c2, int M, double* sol) {
    const int r = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const double ubar = (c1[r] - b2[r]) / c2[0];
    if (k < M) sol[(size_t)r * (M + 1) + k] = fmac(-ubar, q2[k], q1[(size_t)r * M + k]);
    if (k == M) sol[(size_t)r * (M + 1) + M] = ubar;
}

// u[r][:] += z[r][M]
__global__ void k_add_scalar(double* u, size_t len, const double* __restrict__ z, size_t zs, int M) {
    const int r = blockIdx.y;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) u[(size_t)r * len + i] += z[(size_t)r * zs + M];
}

inline unsigned nb(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

// out[r * os] = coef * sum over the grid of g[r] (g: [nrhs][len]); zero when g is null;
// temporaries go to tmp
void grid_sums(ibdl_plan p, int nrhs, const double* g, double coef, double* out, size_t os, std::vector<void*>& tmp,
               hipStream_t st) {
    const size_t len = (size_t)p->nlines * p->n;
    if (!g) {
        for (int r = 0; r < nrhs; ++r) IBDL_HIP_TRY(hipMemsetAsync(out + (size_t)r * os, 0, sizeof(double), st));
        return;
    }
    const int parts = 256;
    double* part = reinterpret_cast<double*>(dev_alloc(tmp, (size_t)nrhs * parts * sizeof(double)));
    hipLaunchKernelGGL(k_gsum_part, dim3(parts, nrhs), dim3(RT), 0, st, g, len, parts, part);
    hipLaunchKernelGGL(k_gsum_final, dim3(nb(nrhs, 64)), dim3(64), 0, st, (const double*)part, parts, nrhs, coef, out,
                       os);
}

// the K pass of the completed operator (IBDL operator plus eta times the single layer)
void completed_K(ibdl_plan p, int nrhs, const double* q, size_t qs, double* out, size_t os, hipStream_t st) {
    PipeIn in;
    in.q_dip = q;
    in.c_dip = 1.0;
    in.q_mono = q;
    in.c_mono = p->eta;
    in.q_stride = qs;
    PipeOut o;
    o.out = out;
    o.out_stride = os;
    o.cA = -1.0;
    o.in = q;
    o.in_stride = qs;
    o.cB = 0.5;
    run_pipeline(p, nrhs, in, o, st);
}

}  // namespace

void completed_apply(ibdl_plan p, int nrhs, const double* z, double* out, hipStream_t st) {
    const int M = p->M;
    const size_t L = (size_t)M + 1;
    completed_K(p, nrhs, z, L, out, L, st);
    hipLaunchKernelGGL(k_add_last, dim3(nb(M, 256), nrhs), dim3(256), 0, st, z, L, out, L, M);
    hipLaunchKernelGGL(k_wsum, dim3(nrhs), dim3(RT), 0, st, z, L, (const double*)p->wgt, M, p->eta, out + M, L);
    IBDL_HIP_TRY(hipGetLastError());
}

void completed_rhs(ibdl_plan p, int nrhs, const double* data, const double* g, double* b, hipStream_t st) {
    const int M = p->M;
    const size_t L = (size_t)M + 1;
    PipeIn in;
    in.grid = g;
    in.c_grid = 1.0;
    PipeOut o;
    o.out = b;
    o.out_stride = L;
    o.cA = -1.0;
    o.in = data;
    o.cB = 1.0;
    run_pipeline(p, nrhs, in, o, st, true);
    double hd = 1.0;
    for (int d = 0; d < p->dim; ++d) hd *= p->h;
    std::vector<void*> tmp;
    grid_sums(p, nrhs, g, hd, b + M, L, tmp, st);
    for (void* t : tmp) dev_free(t);
    IBDL_HIP_TRY(hipGetLastError());
}

void completed_eval_grid(ibdl_plan p, int nrhs, const double* z, const double* g, double* u, hipStream_t st) {
    const int M = p->M;
    const size_t L = (size_t)M + 1;
    PipeIn in;
    in.q_dip = z;
    in.c_dip = -1.0;
    in.q_mono = z;
    in.c_mono = -p->eta;
    in.q_stride = L;
    in.grid = g;
    in.c_grid = 1.0;
    PipeOut o;
    o.u = u;
    run_pipeline(p, nrhs, in, o, st, true);
    const size_t len = (size_t)p->nlines * p->n;
    hipLaunchKernelGGL(k_add_scalar, dim3(nb(len, 256), nrhs), dim3(256), 0, st, u, len, z, L, M);
    IBDL_HIP_TRY(hipGetLastError());
}

int completed_solve(ibdl_plan p, int nrhs, const double* data, const double* g, const ibdl_solve_opts& o,
                    double* sol, double* u, ibdl_solve_info* info, hipStream_t st) {
    const int M = p->M;
    if (!p->ones) {
        p->ones = reinterpret_cast<double*>(dev_alloc(p, (size_t)M * sizeof(double)));
        std::vector<double> h1((size_t)M, 1.0);
        IBDL_HIP_TRY(hipMemcpyAsync(p->ones, h1.data(), (size_t)M * sizeof(double), hipMemcpyHostToDevice, st));
        IBDL_HIP_TRY(hipStreamSynchronize(st));
    }
    if (!p->cq2) {
        // K Q2 = 1 to near FP64 rounding, once per plan; c2 = eta w.Q2
        p->cq2 = reinterpret_cast<double*>(dev_alloc(p, ((size_t)M + 1) * sizeof(double)));
        ibdl_solve_opts o2{1e-13, 50, 1000, nullptr, 0};
        ibdl_solve_info i2{};
        int ov = IBDL_OK;
        p->ks.inst.assign(1, Inst{p, 1, 0});
        p->ks.R = 1;
        solve_set(p->ks, {p->ones}, {nullptr}, {nullptr}, o2, {p->cq2}, &i2, st, &ov);
        if (ov != IBDL_OK) {
            dev_free(p->cq2);
            p->allocs.erase(std::remove(p->allocs.begin(), p->allocs.end(), (void*)p->cq2), p->allocs.end());
            p->cq2 = nullptr;
            throw Error{ov, "the completion's auxiliary solve K Q2 = 1 did not converge"};
        }
        hipLaunchKernelGGL(k_wsum, dim3(1), dim3(RT), 0, st, (const double*)p->cq2, (size_t)M, (const double*)p->wgt, M,
                           p->eta, p->cq2 + M, (size_t)M + 1);
    }
    // K Q1 = U_b - S* D0^-1 g~ for every right-hand side
    std::vector<void*> tmp;
    double* q1 = reinterpret_cast<double*>(dev_alloc(tmp, (size_t)nrhs * M * sizeof(double)));
    double* sc = reinterpret_cast<double*>(dev_alloc(tmp, 2 * (size_t)nrhs * sizeof(double)));
    int overall = IBDL_OK;
    p->ks.inst.assign(1, Inst{p, nrhs, 0});
    p->ks.R = nrhs;
    solve_set(p->ks, {data}, {g}, {nullptr}, o, {q1}, info, st, &overall);
    double hd = 1.0;
    for (int d = 0; d < p->dim; ++d) hd *= p->h;
    hipLaunchKernelGGL(k_wsum, dim3(nrhs), dim3(RT), 0, st, (const double*)q1, (size_t)M, (const double*)p->wgt, M,
                       p->eta, sc, (size_t)1);
    grid_sums(p, nrhs, g, hd, sc + nrhs, 1, tmp, st);
    hipLaunchKernelGGL(k_combine, dim3(nb((size_t)M + 1, 256), nrhs), dim3(256), 0, st, (const double*)q1,
                       (const double*)p->cq2, (const double*)sc, (const double*)(sc + nrhs),
                       (const double*)(p->cq2 + M), M, sol);
    if (u) completed_eval_grid(p, nrhs, sol, g, u, st);
    for (void* t : tmp) dev_free(t);
    IBDL_HIP_TRY(hipGetLastError());
    IBDL_HIP_TRY(hipStreamSynchronize(st));
    return overall;
}

}  // namespace ibdl

// ---------------------------------------------------------------------------
// The IB constraint (single-layer) system, the paper's comparison method
// (Sec. 2.1; Table 1, Table 2): A F = -S* L^-1 S F, right-hand side
// U_b - S* L^-1 g~, grid solution u = L^-1 (g~ - S F), solved by MINRES
// (Paige-Saunders).  A is self-adjoint in <x, y>_W = sum_k w_k x_k y_k (S spreads
// with the point weights), so the Lanczos process runs in that inner product;
// with equal weights it is the plain MINRES of the paper.  All vectors and
// scalars of the iteration stay on the device; the host only looks at the
// per-rhs state between chunks of iterations.
namespace ibdl {

namespace {

enum { MR_DONE = 0, MR_ITERS = 1, MR_STATUS = 2, MR_ACTIVE = 3 };
// per-rhs scalars
enum { S_BETA1, S_BETA, S_OLDB, S_DBAR, S_EPS, S_PHIBAR, S_CS, S_SN, S_ALFA, S_PHI, S_GINV, S_DELTA, S_OLDEPS,
       S_TOL, S_N };

struct MrArgs {
    int R, M, nblk, maxit;
    const double* w;     // [M] point weights
    double *b, *x, *r1, *r2, *v, *y, *wv, *w1, *w2;  // [R][M]
    double* part;        // [R][nblk]
    double* sc;          // [R][S_N]
    int32_t* state;      // [R][4]
};

// block partial of sum_k w_k a_k c_k over this block's points (fixed order)
__device__ __forceinline__ void mr_block_dot(const MrArgs& a, int r, double val) {
    __shared__ double sh[RT];
    sh[threadIdx.x] = val;
    __syncthreads();
    for (int off = RT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.part[(size_t)r * a.nblk + blockIdx.x] = sh[0];
}

__device__ __forceinline__ double mr_sum_parts(const MrArgs& a, int r) {
    double s = 0.0;
    for (int b = 0; b < a.nblk; ++b) s += a.part[(size_t)r * a.nblk + b];
    return s;
}

// x = 0, r1 = r2 = b, wv = w2 = 0; partials of ||b||_W^2
__global__ __launch_bounds__(RT) void k_mr_init(MrArgs a) {
    const int r = blockIdx.y, k = blockIdx.x * RT + threadIdx.x;
    double val = 0.0;
    if (k < a.M) {
        const size_t i = (size_t)r * a.M + k;
        const double bv = a.b[i];
        a.x[i] = 0.0;
        a.r1[i] = bv;
        a.r2[i] = bv;
        a.wv[i] = 0.0;
        a.w2[i] = 0.0;
        val = a.w[k] * bv * bv;
    }
    mr_block_dot(a, r, val);
}

__global__ void k_mr_init_scalars(MrArgs a, double tol) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.R) return;
    double* s = a.sc + (size_t)r * S_N;
    const double beta1 = sqrt(mr_sum_parts(a, r));
    s[S_BETA1] = beta1;
    s[S_BETA] = beta1;
    s[S_OLDB] = 0.0;
    s[S_DBAR] = 0.0;
    s[S_EPS] = 0.0;
    s[S_PHIBAR] = beta1;
    s[S_CS] = -1.0;
    s[S_SN] = 0.0;
    s[S_TOL] = tol;
    int32_t* st = a.state + 4 * r;
    st[MR_DONE] = !(beta1 > 0.0);
    st[MR_ITERS] = 0;
    st[MR_STATUS] = isfinite(beta1) ? IBDL_OK : IBDL_ERR_NUMERIC;
    st[MR_ACTIVE] = 0;
    if (!isfinite(beta1)) st[MR_DONE] = 1;
}

// v = r2 / beta
__global__ __launch_bounds__(RT) void k_mr_v(MrArgs a) {
    const int r = blockIdx.y, k = blockIdx.x * RT + threadIdx.x;
    if (a.state[4 * r + MR_DONE] || k >= a.M) return;
    const size_t i = (size_t)r * a.M + k;
    a.v[i] = a.r2[i] / a.sc[(size_t)r * S_N + S_BETA];
}

// y -= (beta / oldb) r1 (from the second iteration); partials of <v, y>_W
__global__ __launch_bounds__(RT) void k_mr_p1(MrArgs a) {
    const int r = blockIdx.y, k = blockIdx.x * RT + threadIdx.x;
    if (a.state[4 * r + MR_DONE]) return;
    const double* s = a.sc + (size_t)r * S_N;
    const bool later = a.state[4 * r + MR_ITERS] >= 1;
    double val = 0.0;
    if (k < a.M) {
        const size_t i = (size_t)r * a.M + k;
        double yv = a.y[i];
        if (later) yv = fmac(-(s[S_BETA] / s[S_OLDB]), a.r1[i], yv);
        a.y[i] = yv;
        val = a.w[k] * a.v[i] * yv;
    }
    mr_block_dot(a, r, val);
}

__global__ void k_mr_alfa(MrArgs a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.R || a.state[4 * r + MR_DONE]) return;
    a.sc[(size_t)r * S_N + S_ALFA] = mr_sum_parts(a, r);
}

// y -= (alfa / beta) r2; r1 = r2; r2 = y; partials of ||r2||_W^2
__global__ __launch_bounds__(RT) void k_mr_p2(MrArgs a) {
    const int r = blockIdx.y, k = blockIdx.x * RT + threadIdx.x;
    if (a.state[4 * r + MR_DONE]) return;
    const double* s = a.sc + (size_t)r * S_N;
    double val = 0.0;
    if (k < a.M) {
        const size_t i = (size_t)r * a.M + k;
        const double yv = fmac(-(s[S_ALFA] / s[S_BETA]), a.r2[i], a.y[i]);
        a.r1[i] = a.r2[i];
        a.r2[i] = yv;
        val = a.w[k] * yv * yv;
    }
    mr_block_dot(a, r, val);
}

// the Lanczos coefficient beta_{k+1}, the QR update of the tridiagonal matrix by a
// Givens rotation, the residual estimate and the stopping decision
__global__ void k_mr_scal(MrArgs a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.R) return;
    int32_t* st = a.state + 4 * r;
    if (st[MR_DONE]) return;
    double* s = a.sc + (size_t)r * S_N;
    const double beta = sqrt(mr_sum_parts(a, r));
    const double alfa = s[S_ALFA], cs = s[S_CS], sn = s[S_SN], dbar = s[S_DBAR];
    s[S_OLDB] = s[S_BETA];
    s[S_BETA] = beta;
    s[S_OLDEPS] = s[S_EPS];
    s[S_DELTA] = cs * dbar + sn * alfa;
    const double gbar = sn * dbar - cs * alfa;
    s[S_EPS] = sn * beta;
    s[S_DBAR] = -cs * beta;
    const double gamma = hypot(gbar, beta);
    const double c2 = gbar / gamma, s2 = beta / gamma;
    s[S_CS] = c2;
    s[S_SN] = s2;
    s[S_PHI] = c2 * s[S_PHIBAR];
    s[S_PHIBAR] = s2 * s[S_PHIBAR];
    s[S_GINV] = 1.0 / gamma;
    st[MR_ITERS] += 1;
    st[MR_ACTIVE] = 1;
    const double rel = s[S_PHIBAR] / s[S_BETA1];
    if (!isfinite(rel) || !isfinite(gamma)) {
        st[MR_STATUS] = IBDL_ERR_NUMERIC;
        st[MR_DONE] = 1;
        st[MR_ACTIVE] = 0;
    } else if (rel <= s[S_TOL] || !(beta > 0.0)) {
        st[MR_DONE] = 1;
    } else if (st[MR_ITERS] >= a.maxit) {
        st[MR_STATUS] = IBDL_ERR_NOCONV;
        st[MR_DONE] = 1;
    }
}

// w1 = w2; w2 = wv; wv = (v - oldeps w1 - delta w2) / gamma; x += phi wv
__global__ __launch_bounds__(RT) void k_mr_update(MrArgs a) {
    const int r = blockIdx.y, k = blockIdx.x * RT + threadIdx.x;
    if (!a.state[4 * r + MR_ACTIVE]) return;
    const double* s = a.sc + (size_t)r * S_N;
    if (k < a.M) {
        const size_t i = (size_t)r * a.M + k;
        const double w1 = a.w2[i], w2 = a.wv[i];
        const double wn = (a.v[i] - s[S_OLDEPS] * w1 - s[S_DELTA] * w2) * s[S_GINV];
        a.w1[i] = w1;
        a.w2[i] = w2;
        a.wv[i] = wn;
        a.x[i] = fmac(s[S_PHI], wn, a.x[i]);
    }
}

__global__ void k_mr_clear_active(MrArgs a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < a.R) a.state[4 * r + MR_ACTIVE] = 0;
}

}  // namespace

void ibsl_apply(ibdl_plan p, int nrhs, const double* q, double* out, hipStream_t st) {
    PipeIn in;
    in.q_mono = q;
    in.c_mono = 1.0;
    PipeOut o;
    o.out = out;
    o.cA = -1.0;
    run_pipeline(p, nrhs, in, o, st);
}

void ibsl_eval_grid(ibdl_plan p, int nrhs, const double* f, const double* g, double* u, hipStream_t st) {
    PipeIn in;
    in.q_mono = f;
    in.c_mono = -1.0;
    in.grid = g;
    in.c_grid = 1.0;
    PipeOut o;
    o.u = u;
    run_pipeline(p, nrhs, in, o, st, true);
}

int ibsl_solve(ibdl_plan p, int nrhs, const double* data, const double* g, const ibdl_solve_opts& o, double* sol,
               double* u, ibdl_solve_info* info, hipStream_t st) {
    const int M = p->M, R = nrhs;
    const int nblk = (M + RT - 1) / RT;
    std::vector<void*> tmp;
    auto A = [&](size_t n) { return reinterpret_cast<double*>(dev_alloc(tmp, n * sizeof(double))); };
    MrArgs a{};
    a.R = R;
    a.M = M;
    a.nblk = nblk;
    a.maxit = o.maxit;
    a.w = p->wgt;
    const size_t V = (size_t)R * M;
    a.b = A(V);
    a.x = A(V);
    a.r1 = A(V);
    a.r2 = A(V);
    a.v = A(V);
    a.y = A(V);
    a.wv = A(V);
    a.w1 = A(V);
    a.w2 = A(V);
    a.part = A((size_t)R * nblk);
    a.sc = A((size_t)R * S_N);
    a.state = reinterpret_cast<int32_t*>(dev_alloc(tmp, (size_t)R * 4 * sizeof(int32_t)));
    // right-hand side U_b - S* L^-1 g~ (FP64)
    {
        PipeIn in;
        PipeOut po;
        po.out = a.b;
        if (g) {
            in.grid = g;
            in.c_grid = 1.0;
            po.cA = -1.0;
            po.in = data;
            po.cB = 1.0;
            run_pipeline(p, R, in, po, st, true);
        } else {
            IBDL_HIP_TRY(hipMemcpyAsync(a.b, data, V * sizeof(double), hipMemcpyDeviceToDevice, st));
        }
    }
    const dim3 vg(nblk, R), sg((R + 63) / 64);
    hipLaunchKernelGGL(k_mr_init, vg, dim3(RT), 0, st, a);
    hipLaunchKernelGGL(k_mr_init_scalars, sg, dim3(64), 0, st, a, o.tol);
    // the operator pass y = A v, prepared once; converged rhs are skipped by their flag
    PipeIn in;
    in.q_mono = a.v;
    in.c_mono = 1.0;
    in.skip = a.state;
    PipeOut po;
    po.out = a.y;
    po.cA = -1.0;
    std::vector<PassJob> jobs{PassJob{p, R, in, po}};
    std::unique_ptr<PreparedPass> op = prepare_pass(jobs, true);
    std::vector<int32_t> hstate((size_t)R * 4);
    std::vector<double> hsc((size_t)R * S_N);
    int done_iters = 0;
    for (;;) {
        const int chunk = std::min(64, o.maxit - done_iters);
        for (int c = 0; c < chunk; ++c) {
            hipLaunchKernelGGL(k_mr_v, vg, dim3(RT), 0, st, a);
            op->run(0, st);
            hipLaunchKernelGGL(k_mr_p1, vg, dim3(RT), 0, st, a);
            hipLaunchKernelGGL(k_mr_alfa, sg, dim3(64), 0, st, a);
            hipLaunchKernelGGL(k_mr_p2, vg, dim3(RT), 0, st, a);
            hipLaunchKernelGGL(k_mr_scal, sg, dim3(64), 0, st, a);
            hipLaunchKernelGGL(k_mr_update, vg, dim3(RT), 0, st, a);
            hipLaunchKernelGGL(k_mr_clear_active, sg, dim3(64), 0, st, a);
        }
        done_iters += chunk;
        IBDL_HIP_TRY(hipGetLastError());
        IBDL_HIP_TRY(hipMemcpyAsync(hstate.data(), a.state, hstate.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        IBDL_HIP_TRY(hipStreamSynchronize(st));
        bool all = true;
        for (int r = 0; r < R; ++r) all &= hstate[4 * r + MR_DONE] != 0;
        if (all || done_iters >= o.maxit) break;
    }
    IBDL_HIP_TRY(hipMemcpyAsync(hsc.data(), a.sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    IBDL_HIP_TRY(hipMemcpyAsync(sol, a.x, V * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (u) ibsl_eval_grid(p, R, sol, g, u, st);
    IBDL_HIP_TRY(hipStreamSynchronize(st));
    int overall = IBDL_OK;
    for (int r = 0; r < R; ++r) {
        int s = hstate[4 * r + MR_STATUS];
        if (s == IBDL_OK && !hstate[4 * r + MR_DONE]) s = IBDL_ERR_NOCONV;
        if (info) {
            info[r].iters = hstate[4 * r + MR_ITERS];
            const double b1 = hsc[(size_t)r * S_N + S_BETA1];
            info[r].rel_resid_est = b1 > 0.0 ? hsc[(size_t)r * S_N + S_PHIBAR] / b1 : 0.0;
            info[r].rel_resid_true = -1.0;
            info[r].status = s;
            info[r].fp64_applies = 0;
        }
        if (s == IBDL_ERR_NUMERIC) overall = IBDL_ERR_NUMERIC;
        else if (s == IBDL_ERR_NOCONV && overall == IBDL_OK) overall = IBDL_ERR_NOCONV;
    }
    for (void* t : tmp) dev_free(t);
    return overall;
}

}  // namespace ibdl
