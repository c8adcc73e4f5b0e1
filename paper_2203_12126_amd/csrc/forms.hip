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
