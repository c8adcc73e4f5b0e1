// Step 3 of the method (Sec. 4.2, Sec. 5.5): flags of the PDE domain from the
// regularised indicator function (App. D) and the re-interpolation of the grid
// solution near the boundary (App. A).
//
//  * indicator: chi_h = -Delta_0^-1 S~ 1 (one FP64 pass of the grid pipeline with
//    unit strengths and the mean-zero inverse of the Laplacian), shifted so the
//    box corner node lo is 0.  For normals pointing away from the region the
//    boundary encloses chi_h is about 1 there and 0 elsewhere, and the domain is
//    chi_h > 1/2; with normals pointing into it chi_h is about -1 inside and the
//    domain is chi_h > -1/2.  The orientation is the sign of
//    sum_k w_k (X_k - X_0) . n_k (the divergence theorem on the discrete boundary).
//  * fix-up: every domain node whose nearest boundary point lies within m1
//    meshwidths gets u(x_p) = u(x_A) |x_B - x_p| / m2 h + u(x_B) |x_A - x_p| / m2 h,
//    x_A the closest point of the chord between its two nearest boundary points
//    (2-D; the third nearest replaces one of them when the foot of the
//    perpendicular falls outside the chord: the two of the three farthest apart
//    span it), or the nearest boundary point (3-D), with u(x_A) from the
//    boundary values; x_B = x_A + (x_p - x_A)/|x_p - x_A| m2 h, u(x_B) the bi- or
//    trilinear interpolation of the grid solution.  Nodes are found through the
//    plan's cell-sorted points: a candidate mask from the points, then a search
//    of the cell lines around each candidate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "solve.h"

namespace ibdl {

namespace {

constexpr int NF_T = 256;

__global__ void k_fill_ones(double* v, int M) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < M) v[k] = 1.0;
}

__global__ void k_fill_u8(uint8_t* v, size_t n, uint8_t val) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = val;
}

// one block: out[0] = chi value at node 0, out[1] = orientation sign (+1 / -1) of
// sum_k w_k (X_k - X_0) . n_k in caller order (a fixed-order block reduction)
__global__ __launch_bounds__(NF_T) void k_indicator_refs(const double* __restrict__ chi, const double* __restrict__ X,
                                                         const double* __restrict__ nrm, const double* __restrict__ w,
                                                         int M, double* out) {
    __shared__ double sh[NF_T];
    double acc = 0.0;
    for (int k = threadIdx.x; k < M; k += NF_T) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s = fmac(X[3 * k + d] - X[d], nrm[3 * k + d], s);
        acc = fmac(w[k], s, acc);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = NF_T / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = chi[0];
        out[1] = sh[0] > 0.0 ? 1.0 : -1.0;
    }
}

__global__ void k_indicator_flags(double* chi, uint8_t* flags, size_t nn, const double* refs) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const double v = chi[i] - refs[0];
    chi[i] = v;
    flags[i] = v > 0.5 * refs[1] ? 1 : 0;
}

// every node within r cells (per axis, periodic) of a point's cell
__global__ void k_fix_mark(const int32_t* __restrict__ cell, int M, int dim, int n, int r, uint8_t* mask) {
    const int w = 2 * r + 1;
    const int per = dim == 3 ? w * w * w : w * w;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)M * per) return;
    const int s = (int)(id / per), j = (int)(id % per);
    int o[3] = {j % w - r, (j / w) % w - r, dim == 3 ? j / (w * w) - r : 0};
    size_t node = 0, stride = 1;
    for (int d = 0; d < dim; ++d) {
        int c = (cell[3 * s + d] + o[d]) % n;
        if (c < 0) c += n;
        node += (size_t)c * stride;
        stride *= (size_t)n;
    }
    mask[node] = 1;  // every writer stores the same value
}

struct FixArgs {
    const uint8_t* mask;
    const uint8_t* flags;
    const double* u;        // [nrhs][n^dim]
    const double* ub;       // [nrhs][M] caller order
    double* out;            // [nrhs][n^dim]
    int nrhs;
    const double* X;        // [M][3] caller order
    const uint32_t* perm;   // sorted position -> caller index
    const uint32_t* skey;   // cell key of each sorted point
    const int32_t* line_start;
    int dim, n, M;
    double lo0, lo1, lo2, h, L;
    double m1, m2;
    int R;                  // search radius in cells
};

__device__ __forceinline__ double min_image(double v, double L) { return v - L * rint(v / L); }

// keep the three nearest points by (squared distance, caller index)
__device__ __forceinline__ void keep3(double d2, uint32_t k, double (&bd)[3], uint32_t (&bk)[3]) {
    auto less = [](double a, uint32_t ka, double b, uint32_t kb) { return a < b || (a == b && ka < kb); };
    if (!less(d2, k, bd[2], bk[2])) return;
    if (less(d2, k, bd[1], bk[1])) {
        bd[2] = bd[1];
        bk[2] = bk[1];
        if (less(d2, k, bd[0], bk[0])) {
            bd[1] = bd[0];
            bk[1] = bk[0];
            bd[0] = d2;
            bk[0] = k;
        } else {
            bd[1] = d2;
            bk[1] = k;
        }
    } else {
        bd[2] = d2;
        bk[2] = k;
    }
}

// first position in [b, e) of the sorted points whose x cell is >= cx (the points
// of one cell line are sorted by x cell, the key's remainder by n)
__device__ __forceinline__ int lower_cx(const FixArgs& a, int b, int e, int cx) {
    while (b < e) {
        const int mid = (b + e) >> 1;
        if ((int)(a.skey[mid] % (uint32_t)a.n) < cx) b = mid + 1; else e = mid;
    }
    return b;
}

__global__ __launch_bounds__(NF_T) void k_fixup(FixArgs a) {
    const size_t nn = a.dim == 3 ? (size_t)a.n * a.n * a.n : (size_t)a.n * a.n;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const bool cand = a.mask[i] && a.flags[i];
    if (!cand) {
        for (int r = 0; r < a.nrhs; ++r) a.out[(size_t)r * nn + i] = a.u[(size_t)r * nn + i];
        return;
    }
    const int ix = (int)(i % a.n), iy = (int)((i / a.n) % a.n), iz = a.dim == 3 ? (int)(i / ((size_t)a.n * a.n)) : 0;
    const double xp[3] = {a.lo0 + a.h * ix, a.lo1 + a.h * iy, a.dim == 3 ? a.lo2 + a.h * iz : 0.0};
    double bd[3] = {INFINITY, INFINITY, INFINITY};
    uint32_t bk[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
    const int R = a.R;
    // cell lines within R of the node, each visited once also where 2R+1 >= n
    const bool wrapall = 2 * R + 1 >= a.n;
    const int wl = wrapall ? a.n : 2 * R + 1;
    const int nz = a.dim == 3 ? wl : 1;
    for (int dz = 0; dz < nz; ++dz) {
        int cz = 0;
        if (a.dim == 3) {
            cz = wrapall ? dz : (iz - R + dz) % a.n;
            if (cz < 0) cz += a.n;
        }
        for (int dy = 0; dy < wl; ++dy) {
            int cy = wrapall ? dy : (iy - R + dy) % a.n;
            if (cy < 0) cy += a.n;
            const int line = cz * a.n + cy;
            const int b = a.line_start[line], e = a.line_start[line + 1];
            if (b == e) continue;
            // x cells ix-R .. ix+R, as one or two ranges of the periodic axis
            int lo = ix - R, hi = ix + R;
            int r0[2] = {0, 0}, r1[2] = {-1, -1};
            if (2 * R + 1 >= a.n) {
                r0[0] = 0;
                r1[0] = a.n - 1;
            } else if (lo < 0) {
                r0[0] = 0; r1[0] = hi;
                r0[1] = lo + a.n; r1[1] = a.n - 1;
            } else if (hi >= a.n) {
                r0[0] = lo; r1[0] = a.n - 1;
                r0[1] = 0; r1[1] = hi - a.n;
            } else {
                r0[0] = lo; r1[0] = hi;
            }
            for (int q = 0; q < 2; ++q) {
                if (r1[q] < r0[q]) continue;
                const int s0 = lower_cx(a, b, e, r0[q]);
                const int s1 = lower_cx(a, s0, e, r1[q] + 1);
                for (int s = s0; s < s1; ++s) {
                    const uint32_t k = a.perm[s];
                    double d2 = 0.0;
                    for (int d = 0; d < a.dim; ++d) {
                        const double v = min_image(a.X[3 * k + d] - xp[d], a.L);
                        d2 = fmac(v, v, d2);
                    }
                    keep3(d2, k, bd, bk);
                }
            }
        }
    }
    const double d1 = sqrt(bd[0]);
    if (bk[0] == 0xffffffffu || !(d1 <= a.m1 * a.h)) {
        for (int r = 0; r < a.nrhs; ++r) a.out[(size_t)r * nn + i] = a.u[(size_t)r * nn + i];
        return;
    }
    // x_A and the boundary values' weights
    double xa[3] = {0.0, 0.0, 0.0};
    uint32_t ka = bk[0], kb = bk[0];
    double wa = 1.0, wb = 0.0;
    const uint32_t kNone = 0xffffffffu;
    if (a.dim == 2 && bk[1] != kNone) {
        double x1[2], x2[2], x3[2];
        for (int d = 0; d < 2; ++d) {
            x1[d] = xp[d] + min_image(a.X[3 * bk[0] + d] - xp[d], a.L);
            x2[d] = xp[d] + min_image(a.X[3 * bk[1] + d] - xp[d], a.L);
        }
        uint32_t k1 = bk[0], k2 = bk[1];
        double e0 = x1[0] - x2[0], e1 = x1[1] - x2[1];
        double t = fmac(xp[0] - x2[0], e0, (xp[1] - x2[1]) * e1) / fmac(e0, e0, e1 * e1);
        if ((t < 0.0 || t > 1.0) && bk[2] != kNone) {
            for (int d = 0; d < 2; ++d) x3[d] = xp[d] + min_image(a.X[3 * bk[2] + d] - xp[d], a.L);
            auto sq = [](const double* p, const double* q) {
                const double u0 = p[0] - q[0], u1 = p[1] - q[1];
                return fmac(u0, u0, u1 * u1);
            };
            // the two of the three farthest apart (first of equal pairs in the order 12, 13, 23)
            const double s12 = sq(x1, x2), s13 = sq(x1, x3), s23 = sq(x2, x3);
            if (s13 > s12 && s13 >= s23) {
                x2[0] = x3[0]; x2[1] = x3[1]; k2 = bk[2];
            } else if (s23 > s12 && s23 > s13) {
                x1[0] = x2[0]; x1[1] = x2[1]; k1 = bk[1];
                x2[0] = x3[0]; x2[1] = x3[1]; k2 = bk[2];
            }
            e0 = x1[0] - x2[0];
            e1 = x1[1] - x2[1];
            t = fmac(xp[0] - x2[0], e0, (xp[1] - x2[1]) * e1) / fmac(e0, e0, e1 * e1);
        }
        t = fmin(1.0, fmax(0.0, t));
        xa[0] = fmac(t, e0, x2[0]);
        xa[1] = fmac(t, e1, x2[1]);
        const double le = sqrt(fmac(e0, e0, e1 * e1));
        const double da2 = sqrt((xa[0] - x2[0]) * (xa[0] - x2[0]) + (xa[1] - x2[1]) * (xa[1] - x2[1]));
        const double da1 = sqrt((xa[0] - x1[0]) * (xa[0] - x1[0]) + (xa[1] - x1[1]) * (xa[1] - x1[1]));
        ka = k1;
        kb = k2;
        wa = da2 / le;  // weight of U_b(x1)
        wb = da1 / le;  // weight of U_b(x2)
    } else {
        // 3-D, or a 2-D node with a single point in reach: x_A is the nearest point
        for (int d = 0; d < a.dim; ++d) xa[d] = xp[d] + min_image(a.X[3 * bk[0] + d] - xp[d], a.L);
    }
    double dp2 = 0.0;
    for (int d = 0; d < a.dim; ++d) dp2 = fmac(xp[d] - xa[d], xp[d] - xa[d], dp2);
    const double dp = sqrt(dp2);
    // x_B and its bi-/trilinear stencil
    double cw = 0.0, cb = 0.0;
    size_t cidx[8];
    double cwt[8];
    int nc = 0;
    if (dp > 0.0) {
        double xb[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < a.dim; ++d) xb[d] = xa[d] + (xp[d] - xa[d]) / dp * (a.m2 * a.h);
        double dab2 = 0.0, dbp2 = 0.0;
        for (int d = 0; d < a.dim; ++d) {
            dab2 = fmac(xb[d] - xa[d], xb[d] - xa[d], dab2);
            dbp2 = fmac(xb[d] - xp[d], xb[d] - xp[d], dbp2);
        }
        const double dab = sqrt(dab2), dbp = sqrt(dbp2);
        cw = dbp / dab;  // weight of u(x_A)
        cb = dp / dab;   // weight of u(x_B)
        const double lo[3] = {a.lo0, a.lo1, a.lo2};
        long long fl[3];
        double fr[3];
        for (int d = 0; d < a.dim; ++d) {
            const double t = (xb[d] - lo[d]) / a.h;
            const double f = floor(t);
            fl[d] = (long long)f;
            fr[d] = t - f;
        }
        nc = 1 << a.dim;
        for (int c = 0; c < nc; ++c) {
            double w = 1.0;
            size_t node = 0, stride = 1;
            for (int d = 0; d < a.dim; ++d) {
                const int bit = (c >> d) & 1;
                w *= bit ? fr[d] : 1.0 - fr[d];
                long long q = (fl[d] + bit) % a.n;
                if (q < 0) q += a.n;
                node += (size_t)q * stride;
                stride *= (size_t)a.n;
            }
            cidx[c] = node;
            cwt[c] = w;
        }
    }
    for (int r = 0; r < a.nrhs; ++r) {
        const double* ubr = a.ub + (size_t)r * a.M;
        const double ua = ka != kb ? (ubr[ka] * wa + ubr[kb] * wb) : ubr[ka];
        double val = ua;
        if (dp > 0.0) {
            const double* ur = a.u + (size_t)r * nn;
            double ubv = 0.0;
            for (int c = 0; c < nc; ++c) ubv += cwt[c] * ur[cidx[c]];
            val = ua * cw + ubv * cb;
        }
        a.out[(size_t)r * nn + i] = val;
    }
}

inline int nb(size_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void nearfix_indicator(ibdl_plan p, double* chi, uint8_t* flags, hipStream_t st) {
    if (!p->ones) {
        p->ones = reinterpret_cast<double*>(dev_alloc(p, (size_t)p->M * sizeof(double)));
        hipLaunchKernelGGL(k_fill_ones, dim3(nb(p->M, 256)), dim3(256), 0, st, p->ones, p->M);
    }
    if (!p->fix_refs) p->fix_refs = reinterpret_cast<double*>(dev_alloc(p, 2 * sizeof(double)));
    PipeIn in;
    in.q_dip = p->ones;
    in.c_dip = -1.0;
    in.alpha_zero = true;
    PipeOut out;
    out.u = chi;
    run_pipeline(p, 1, in, out, st, true);
    const size_t nn = (size_t)p->nlines * p->n;
    hipLaunchKernelGGL(k_indicator_refs, dim3(1), dim3(NF_T), 0, st, chi, p->X, p->nrm, p->wgt, p->M, p->fix_refs);
    hipLaunchKernelGGL(k_indicator_flags, dim3(nb(nn, 256)), dim3(256), 0, st, chi, flags, nn,
                       (const double*)p->fix_refs);
    IBDL_HIP_TRY(hipGetLastError());
}

void nearfix_fixup(ibdl_plan p, int nrhs, const double* u, const double* ub, const uint8_t* flags, double m1,
                   double m2, double* uout, hipStream_t st) {
    const size_t nn = (size_t)p->nlines * p->n;
    if (!p->fix_mask) p->fix_mask = reinterpret_cast<uint8_t*>(dev_alloc(p, nn));
    const int rmark = (int)std::ceil(m1) + 1;
    // 2-D: the second and third nearest points lie within a few point spacings of the nearest
    const int rsearch = p->dim == 2 ? (int)std::ceil(m1) + 5 : rmark;
    hipLaunchKernelGGL(k_fill_u8, dim3(nb(nn, 256)), dim3(256), 0, st, p->fix_mask, nn, (uint8_t)0);
    const int w = 2 * rmark + 1;
    const long long marks = (long long)p->M * (p->dim == 3 ? (long long)w * w * w : (long long)w * w);
    hipLaunchKernelGGL(k_fix_mark, dim3((unsigned)((marks + 255) / 256)), dim3(256), 0, st, p->cell, p->M, p->dim,
                       p->n, rmark, p->fix_mask);
    FixArgs a{};
    a.mask = p->fix_mask;
    a.flags = flags;
    a.u = u;
    a.ub = ub;
    a.out = uout;
    a.nrhs = nrhs;
    a.X = p->X;
    a.perm = p->perm;
    a.skey = p->skey;
    a.line_start = p->line_start;
    a.dim = p->dim;
    a.n = p->n;
    a.M = p->M;
    a.lo0 = p->lo[0];
    a.lo1 = p->lo[1];
    a.lo2 = p->lo[2];
    a.h = p->h;
    a.L = p->length;
    a.m1 = m1;
    a.m2 = m2;
    a.R = rsearch;
    hipLaunchKernelGGL(k_fixup, dim3(nb(nn, NF_T)), dim3(NF_T), 0, st, a);
    IBDL_HIP_TRY(hipGetLastError());
}

}  // namespace ibdl
