// Unpreconditioned restarted GMRES on the boundary density (Sec. 5.3), FP64 on
// the device, for a set of right-hand sides that may belong to different plans
// (different boundary sizes M, grids, boundary conditions, precisions).
//
// Arnoldi step j of right-hand side r:  w = A v_j (one pass of the operator, whose
// finishing kernel also forms the block partial sums of <w, v_i>), then
// h_ij = <w, v_i> and w -= sum_i h_ij v_i twice (classical Gram-Schmidt applied
// twice; the first pass also sums ||w||^2 so that h_{j+1,j} needs no further
// reduction), v_{j+1} = w / h_{j+1,j}; the previous Givens rotations
// are applied to column j, a new rotation zeroes h_{j+1,j}, and the rotated
// right-hand side g gives the residual estimate |g_{j+1}|.  Every inner product is
// a two-level block reduction in a fixed order over the rhs's own blocks, so a
// right-hand side's arithmetic does not depend on which others share the launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <tuple>
#include <vector>

#include "solve.h"

namespace ibdl {

__device__ __forceinline__ int imin_d(int a, int b) { return a < b ? a : b; }

constexpr int GT = 256;  // threads per block = vector elements per block (= points per finishing block)

enum { ST_DONE = 0, ST_ITERS = 1, ST_STATUS = 2, ST_J = 3 };

// relative residual at which the first FP32-operator solve of a mixed instance stops
constexpr double kMixedFirstTol = 1e-6;

// Device view of the Krylov state of R right-hand sides.
struct KArgs {
    int R, m;
    const int32_t* Mr;
    const size_t* voff;
    const size_t* xoff;
    double* V;
    double* part;       // [R][nblk][m+2] (two banks: part and part2)
    double* part2;
    size_t pstride;     // per rhs
    double* hcol;       // [R][m+2]
    double* H;          // [R][m][m+1]: column j at H + j*(m+1)
    double* cs;         // [R][m]
    double* sn;
    double* g;          // [R][m+1]
    double* y;          // [R][m]
    double* bnorm;      // [R]
    double* resid;      // [R]
    double* nrm;        // [R]
    const double* tolv; // [R] tolerance relative to ||b_r||
    int32_t* state;     // [R][4]
    const int32_t* skip;
    const int32_t* maxv;  // [R] Arnoldi steps each rhs may take in the current Krylov run
    const int32_t* jp;  // base of the Arnoldi step index in device memory (added to the
                        // launch argument), or null: the launch argument alone
    int32_t* jcur;      // the step index that replayed steps read; reset with each cycle
};

__device__ __forceinline__ int nblocks_of(int M) { return (M + GT - 1) / GT; }

// s = sum over b < nb of p[b * stride] in b order, the loads issued eight at a time
__device__ __forceinline__ double sum_strided(const double* __restrict__ p, int nb, size_t stride) {
    double s = 0.0;
    int b = 0;
    for (; b + 8 <= nb; b += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = p[(size_t)(b + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += t[u];
    }
    for (; b < nb; ++b) s += p[(size_t)b * stride];
    return s;
}

// Block sums of nv per-thread values at once: each wave reduces its values with
// cross-lane shuffles, one LDS write per wave and value, one barrier, then
// thread i adds the wave totals of value i (fixed order).  out[i] valid in
// threads i < nv after the call.
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
    if ((int)threadIdx.x < nv) {
        double t = 0.0;
        for (int ww = 0; ww < GT / 64; ++ww) t += sh[ww * MAXV + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// block partial sums of x^2 (pool vectors) into part[r][b]
__global__ __launch_bounds__(GT) void k_sumsq(KArgs a, const double* __restrict__ pool) {
    __shared__ double sh[GT / 64];
    __shared__ double o1[1];
    const int r = blockIdx.y, M = a.Mr[r];
    if ((int)blockIdx.x >= nblocks_of(M)) return;
    const int m = blockIdx.x * GT + threadIdx.x;
    double v[1] = {0.0};
    if (m < M) {
        const double x = pool[a.xoff[r] + m];
        v[0] = x * x;
    }
    block_multi_sum<1>(v, 1, sh, o1);
    if (threadIdx.x == 0) a.part[(size_t)r * a.pstride + blockIdx.x] = o1[0];
}

// nrm[r] = sqrt of the summed block partials of k_sumsq
__global__ void k_norms(KArgs a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.R) return;
    const int nb = nblocks_of(a.Mr[r]);
    const double s = sum_strided(a.part + (size_t)r * a.pstride, nb, 1);
    a.nrm[r] = sqrt(s);
}

__global__ void k_set_bnorm(KArgs a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.R) return;
    const int nb = nblocks_of(a.Mr[r]);
    const double s = sum_strided(a.part + (size_t)r * a.pstride, nb, 1);
    a.bnorm[r] = sqrt(s);
    a.state[4 * r + ST_DONE] = a.skip[r];
    a.state[4 * r + ST_ITERS] = 0;
    a.state[4 * r + ST_STATUS] = isfinite(s) ? IBDL_OK : IBDL_ERR_NUMERIC;
    a.state[4 * r + ST_J] = 0;
    if (r == 0 && a.jcur) *a.jcur = 0;
}

// start a cycle: v_0 = r / ||r||, g = (||r||, 0, ...); rhs already done are left alone
__global__ __launch_bounds__(GT) void k_init_cycle(KArgs a, const double* __restrict__ rpool) {
    const int r = blockIdx.y, M = a.Mr[r];
    const int nb = nblocks_of(M);
    int32_t* st = a.state + 4 * r;
    if (st[ST_DONE] || (int)blockIdx.x >= nb) return;
    const double s = sum_strided(a.part + (size_t)r * a.pstride, nb, 1);
    const double beta = sqrt(s);
    const double bn = a.bnorm[r];
    const bool done = !(bn > 0.0) || beta <= a.tolv[r] * bn || !(beta > 0.0);
    const double inv = (beta > 0.0) ? 1.0 / beta : 0.0;
    const int m = blockIdx.x * GT + threadIdx.x;
    if (m < M) a.V[a.voff[r] + m] = rpool[a.xoff[r] + m] * inv;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double* g = a.g + (size_t)r * (a.m + 1);
        g[0] = beta;
        for (int i = 1; i <= a.m; ++i) g[i] = 0.0;
        a.resid[r] = bn > 0.0 ? beta / bn : 0.0;
        st[ST_J] = 0;
        if (!isfinite(s)) st[ST_STATUS] = IBDL_ERR_NUMERIC;
        if (done || !isfinite(s)) st[ST_DONE] = 1;
    }
}

// First Gram-Schmidt pass of Arnoldi step j: h1 = sum of the block partials of
// <w, v_i> (left by the operator's finishing kernel), w' = w - V h1, and the
// block partials of <w', v_i> (i <= j) and of ||w'||^2 (slot j+1).
__global__ __launch_bounds__(GT) void k_orth(KArgs a, int j) {
    __shared__ double hs[256];
    __shared__ double msh[(GT / 64) * 16];
    __shared__ double mout[16];
    if (a.jp) j += *a.jp;
    const int r = blockIdx.y, M = a.Mr[r];
    const int nb = nblocks_of(M);
    if (a.state[4 * r + ST_DONE] || (int)blockIdx.x >= nb) return;
    const double* pin = a.part + (size_t)r * a.pstride;
    double* pout = a.part2 + (size_t)r * a.pstride;
    for (int vi = threadIdx.x; vi <= j; vi += GT) {
        const double s = sum_strided(pin + vi, nb, (size_t)(a.m + 2));
        hs[vi] = s;
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int vi = threadIdx.x; vi <= j; vi += GT) a.hcol[(size_t)r * (a.m + 2) + vi] = hs[vi];
    double* V = a.V + a.voff[r];
    double* w = V + (size_t)(j + 1) * M;
    const int m = blockIdx.x * GT + threadIdx.x;
    double wl = 0.0;
    if (m < M) {
        // w -= sum_i h_i v_i in index order, loads issued 8 at a time
        double acc = w[m];
        int vi = 0;
        for (; vi + 8 <= j + 1; vi += 8) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = V[(size_t)(vi + u) * M + m];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = fmac(-hs[vi + u], t[u], acc);
        }
        for (; vi <= j; ++vi) acc = fmac(-hs[vi], V[(size_t)vi * M + m], acc);
        wl = acc;
        w[m] = acc;
    }
    // <w', v_i> for i <= j and ||w'||^2, 16 at a time
    const int nvt = j + 2;
    for (int v0 = 0; v0 < nvt; v0 += 16) {
        const int nv = imin_d(16, nvt - v0);
        double acc[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int vi = v0 + u;
            acc[u] = (u < nv && m < M) ? (vi <= j ? V[(size_t)vi * M + m] : wl) * wl : 0.0;
        }
        block_multi_sum<16>(acc, nv, msh, mout);
        if ((int)threadIdx.x < nv) pout[(size_t)blockIdx.x * (a.m + 2) + v0 + threadIdx.x] = mout[threadIdx.x];
    }
}

// Second Gram-Schmidt pass and normalisation of Arnoldi step j: h2 = sum of the
// partials of <w', v_i>, h_{j+1,j} = sqrt(||w'||^2 - ||h2||^2) (= ||w' - V h2||
// for orthonormal V), v_{j+1} = (w' - V h2) / h_{j+1,j}; block 0 applies the
// previous Givens rotations to the column h1 + h2, forms the new one and updates
// the residual estimate and the state.
__global__ __launch_bounds__(GT) void k_orth_final(KArgs a, int j) {
    __shared__ double hs[256];
    __shared__ double hn_s[2];
    __shared__ double hc_s[256], cs_s[256], sn_s[256];
    if (a.jp) j += *a.jp;
    const int r = blockIdx.y, M = a.Mr[r];
    const int nb = nblocks_of(M);
    int32_t* st = a.state + 4 * r;
    if (st[ST_DONE] || (int)blockIdx.x >= nb) return;
    const double* pin = a.part2 + (size_t)r * a.pstride;
    for (int vi = threadIdx.x; vi <= j + 1; vi += GT) {
        const double s = sum_strided(pin + vi, nb, (size_t)(a.m + 2));
        hs[vi] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double q = 0.0;
        for (int vi = 0; vi <= j; ++vi) q = fmac(hs[vi], hs[vi], q);
        const double d = hs[j + 1] - q;
        hn_s[0] = d > 0.0 ? sqrt(d) : 0.0;
        hn_s[1] = hs[j + 1];
    }
    __syncthreads();
    const double hn = hn_s[0];
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    double* V = a.V + a.voff[r];
    double* w = V + (size_t)(j + 1) * M;
    const int m = blockIdx.x * GT + threadIdx.x;
    if (m < M) {
        double acc = w[m];
        int vi = 0;
        for (; vi + 8 <= j + 1; vi += 8) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = V[(size_t)(vi + u) * M + m];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = fmac(-hs[vi + u], t[u], acc);
        }
        for (; vi <= j; ++vi) acc = fmac(-hs[vi], V[(size_t)vi * M + m], acc);
        w[m] = acc * inv;
    }
    if (blockIdx.x != 0) return;
    // the column h1 + h2 and the previous rotations, loaded in parallel
    const double* hc = a.hcol + (size_t)r * (a.m + 2);
    double* cs = a.cs + (size_t)r * a.m;
    double* sn = a.sn + (size_t)r * a.m;
    for (int i = threadIdx.x; i <= j; i += GT) {
        hc_s[i] = hc[i] + hs[i];
        if (i < j) {
            cs_s[i] = cs[i];
            sn_s[i] = sn[i];
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double* Hj = a.H + (size_t)r * a.m * (a.m + 1) + (size_t)j * (a.m + 1);
    double* g = a.g + (size_t)r * (a.m + 1);
    hc_s[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = fmac(cs_s[i], hc_s[i], sn_s[i] * hc_s[i + 1]);
        hc_s[i + 1] = fmac(-sn_s[i], hc_s[i], cs_s[i] * hc_s[i + 1]);
        hc_s[i] = t;
    }
    const double den = hypot(hc_s[j], hc_s[j + 1]);
    const double c = den > 0.0 ? hc_s[j] / den : 1.0;
    const double sv = den > 0.0 ? hc_s[j + 1] / den : 0.0;
    cs[j] = c;
    sn[j] = sv;
    for (int i = 0; i < j; ++i) Hj[i] = hc_s[i];
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sv * gj;
    g[j] = c * gj;
    const double res = fabs(sv * gj) / a.bnorm[r];
    a.resid[r] = res;
    st[ST_ITERS] += 1;
    st[ST_J] = j + 1;
    if (!isfinite(res) || !isfinite(hn_s[1])) {
        st[ST_STATUS] = IBDL_ERR_NUMERIC;
        st[ST_DONE] = 1;
    } else if (res <= a.tolv[r] || !(hn > 0.0) || st[ST_ITERS] >= a.maxv[r]) {
        st[ST_DONE] = 1;
    }
}

// y = R^-1 g over the steps of the current cycle (one block per rhs; the
// triangle is staged in LDS when it fits)
constexpr int BS_T = 64;
constexpr int BS_LDS = 4096;  // doubles
__global__ __launch_bounds__(BS_T) void k_backsolve(KArgs a) {
    __shared__ double Rs[BS_LDS];
    __shared__ double gs[256], ys[256];
    const int r = blockIdx.x;
    const int jr = a.state[4 * r + ST_J];
    const double* H = a.H + (size_t)r * a.m * (a.m + 1);
    const double* g = a.g + (size_t)r * (a.m + 1);
    double* y = a.y + (size_t)r * a.m;
    const bool lds = jr * jr <= BS_LDS;
    for (int i = threadIdx.x; i < jr; i += BS_T) gs[i] = g[i];
    if (lds)
        for (int e = threadIdx.x; e < jr * jr; e += BS_T) {
            const int k = e / jr, i = e % jr;  // column k, row i
            Rs[e] = i <= k ? H[(size_t)k * (a.m + 1) + i] : 0.0;
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = jr - 1; i >= 0; --i) {
            double t = gs[i];
            for (int k = i + 1; k < jr; ++k) t -= (lds ? Rs[k * jr + i] : H[(size_t)k * (a.m + 1) + i]) * ys[k];
            const double d = lds ? Rs[i * jr + i] : H[(size_t)i * (a.m + 1) + i];
            ys[i] = d != 0.0 ? t / d : 0.0;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < jr; i += BS_T) y[i] = ys[i];
}

// x += V[0..jr) y
__global__ __launch_bounds__(GT) void k_update_x(KArgs a, double* xpool) {
    __shared__ double ys[256];
    const int r = blockIdx.y, M = a.Mr[r];
    const int jr = a.state[4 * r + ST_J];
    if (jr == 0 || (int)blockIdx.x * GT >= M) return;
    for (int i = threadIdx.x; i < jr; i += GT) ys[i] = a.y[(size_t)r * a.m + i];
    __syncthreads();
    const int m = blockIdx.x * GT + threadIdx.x;
    if (m >= M) return;
    const double* V = a.V + a.voff[r];
    double acc = xpool[a.xoff[r] + m];
    int vi = 0;
    for (; vi + 8 <= jr; vi += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = V[(size_t)(vi + u) * M + m];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fmac(ys[vi + u], t[u], acc);
    }
    for (; vi < jr; ++vi) acc = fmac(ys[vi], V[(size_t)vi * M + m], acc);
    xpool[a.xoff[r] + m] = acc;
}

// the device-side step index of replayed iterations
__global__ void k_set_j(int32_t* jp, int v) { *jp = v; }
__global__ void k_add_j(int32_t* jp, int c) { *jp += c; }

__global__ void k_reset_j(KArgs a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < a.R) a.state[4 * r + ST_J] = 0;
    if (r == 0) *a.jcur = 0;
}

// pool vectors of the rhs not skipped: op 0: dst = 0, op 1: dst += src
__global__ __launch_bounds__(GT) void k_pool_op(KArgs a, int op, double* dst, const double* src) {
    const int r = blockIdx.y, M = a.Mr[r];
    const int m = blockIdx.x * GT + threadIdx.x;
    if (m >= M || a.skip[r]) return;
    const size_t i = a.xoff[r] + m;
    if (op == 0) dst[i] = 0.0;
    else dst[i] += src[i];
}

// copies of several device vectors in one launch (block row y: job y)
struct CopyJob {
    double* dst;
    const double* src;
    int64_t n;
};
__global__ __launch_bounds__(256) void k_copy_multi(const CopyJob* __restrict__ jobs) {
    const CopyJob jb = jobs[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < jb.n; i += (int64_t)gridDim.x * 256)
        jb.dst[i] = jb.src[i];
}

// ------------------------------------------------------------------ host
// the copies as one launch (its table through the set's arena), or one by one
// when there are only a few
static void copy_multi(KrylovSet& ks, const std::vector<CopyJob>& jobs, hipStream_t st) {
    if (jobs.size() <= 2) {
        for (const CopyJob& j : jobs)
            IBDL_HIP_TRY(hipMemcpyAsync(j.dst, j.src, (size_t)j.n * sizeof(double), hipMemcpyDeviceToDevice, st));
        return;
    }
    int64_t maxn = 1;
    for (const CopyJob& j : jobs) maxn = std::max(maxn, j.n);
    const auto* d = reinterpret_cast<const CopyJob*>(arena_put(*ks.arena, jobs.data(), jobs.size() * sizeof(CopyJob), st));
    const int bx = (int)std::min<int64_t>(64, (maxn + 255) / 256);
    hipLaunchKernelGGL(k_copy_multi, dim3(bx, (unsigned)jobs.size()), dim3(256), 0, st, d);
    IBDL_HIP_TRY(hipGetLastError());
}

void free_krylov(KWork& k) {
    // no replay is in flight here: a solve task waits for its replays before it ends
    for (hipGraphExec_t& g : k.gexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    k.graph_valid = k.op_ran = false;
    k.op.reset();
    k.op_key.clear();
    arena_free(k.op_arena);
    for (void* p : k.mem) dev_free(p);
    k.mem.clear();
    pinned_put(k.host_pinned);
    k.host_pinned = nullptr;
    k.cap_m = 0;
    k.R = 0;
    k.layout.clear();
}

static void ensure_krylov(KrylovSet& ks, int m) {
    KWork& k = ks.w;
    std::vector<std::pair<ibdl_plan, int>> layout;
    for (const Inst& in : ks.inst) layout.emplace_back(in.p, in.nrhs);
    if (k.cap_m >= m && layout == k.layout) return;
    m = std::max(m, k.layout == layout ? k.cap_m : 0);
    free_krylov(k);
    const int R = ks.R;
    size_t vtot = 0, xtot = 0;
    int maxM = 1;
    std::vector<int32_t> Mr(R);
    std::vector<size_t> voff(R), xoff(R);
    for (const Inst& in : ks.inst)
        for (int q = 0; q < in.nrhs; ++q) {
            const int r = in.r0 + q;
            Mr[r] = in.p->M;
            voff[r] = vtot;
            xoff[r] = xtot;
            vtot += (size_t)(m + 1) * in.p->M;
            xtot += (size_t)in.p->M;
            maxM = std::max(maxM, in.p->M);
        }
    const int nblk = (maxM + GT - 1) / GT;
    auto A = [&](size_t n) { return reinterpret_cast<double*>(dev_alloc(k.mem, std::max<size_t>(n, 1) * 8)); };
    k.V = A(vtot);
    k.H = A((size_t)R * m * (m + 1));
    k.cs = A((size_t)R * m);
    k.sn = A((size_t)R * m);
    k.g = A((size_t)R * (m + 1));
    k.y = A((size_t)R * m);
    k.partial = A((size_t)R * nblk * (m + 2) * 2);
    k.hcol = A((size_t)R * (m + 2));
    k.bnorm = A(R);
    // residual estimates [R] followed by the state [R][4]: one snapshot copy
    k.resid = A(R + 2 * (size_t)R);
    k.state = reinterpret_cast<int32_t*>(k.resid + R);
    k.tolv = A(R);
    k.nrm = A(R);
    k.b = A(xtot);
    k.x = A(xtot);
    k.r = A(xtot);
    k.rr = A(xtot);
    k.d = A(xtot);
    // skip flags [R] followed by the per-rhs step budgets [R]: one copy per Krylov run
    k.skip = reinterpret_cast<int32_t*>(dev_alloc(k.mem, 2 * (size_t)R * sizeof(int32_t)));
    k.jcur = reinterpret_cast<int32_t*>(dev_alloc(k.mem, sizeof(int32_t)));
    k.Mr = reinterpret_cast<int32_t*>(dev_alloc(k.mem, (size_t)R * sizeof(int32_t)));
    k.voff = reinterpret_cast<size_t*>(dev_alloc(k.mem, (size_t)R * sizeof(size_t)));
    k.xoff = reinterpret_cast<size_t*>(dev_alloc(k.mem, (size_t)R * sizeof(size_t)));
    // stream-ordered allocations: fill them on the same stream, from host memory
    // that stays valid until the copies are done
    const hipStream_t ast = alloc_stream();
    IBDL_HIP_TRY(hipMemcpyAsync(k.Mr, Mr.data(), R * sizeof(int32_t), hipMemcpyHostToDevice, ast));
    IBDL_HIP_TRY(hipMemcpyAsync(k.voff, voff.data(), R * sizeof(size_t), hipMemcpyHostToDevice, ast));
    IBDL_HIP_TRY(hipMemcpyAsync(k.xoff, xoff.data(), R * sizeof(size_t), hipMemcpyHostToDevice, ast));
    IBDL_HIP_TRY(hipStreamSynchronize(ast));
    // host staging: tolerances, skip flags, state, residuals, norms
    k.host_pinned = pinned_get((size_t)R * (5 * 8 + 10 * 4) + 64);  // the Staging layout
    k.cap_m = m;
    k.R = R;
    k.nblk = nblk;
    k.hvoff = voff;
    k.hxoff = xoff;
    k.layout = layout;
}

static KArgs kargs(KrylovSet& ks, int m) {
    KWork& k = ks.w;
    KArgs a{};
    a.R = ks.R;
    a.m = m;
    a.Mr = k.Mr;
    a.voff = k.voff;
    a.xoff = k.xoff;
    a.V = k.V;
    a.part = k.partial;
    a.pstride = (size_t)k.nblk * (m + 2);
    a.part2 = k.partial + (size_t)ks.R * a.pstride;
    a.hcol = k.hcol;
    a.H = k.H;
    a.cs = k.cs;
    a.sn = k.sn;
    a.g = k.g;
    a.y = k.y;
    a.bnorm = k.bnorm;
    a.resid = k.resid;
    a.nrm = k.nrm;
    a.tolv = k.tolv;
    a.state = k.state;
    a.skip = k.skip;
    a.maxv = k.skip + ks.R;
    a.jp = nullptr;
    a.jcur = k.jcur;
    return a;
}

// host staging: tolerances, skip flags, norms of b, norms of other pools, and two
// alternating snapshots of the per-rhs residual estimates and state (each laid out
// as on the device: [R] doubles, then [R][4] int32)
struct Staging {
    double* tol;
    double* bn;
    double* nrm;
    double* resid[2];
    int32_t* state[2];
    int32_t* skip;   // [R] skip flags, then [R] step budgets (as on the device)
};
static Staging staging(KWork& k, int R) {
    double* d = reinterpret_cast<double*>(k.host_pinned);
    Staging s;
    s.tol = d;
    s.bn = d + R;
    s.nrm = d + 2 * R;
    for (int b = 0; b < 2; ++b) {
        s.resid[b] = d + 3 * R + b * 3 * R;
        s.state[b] = reinterpret_cast<int32_t*>(s.resid[b] + R);
    }
    s.skip = reinterpret_cast<int32_t*>(d + 9 * R);
    return s;
}

GroupedPass prepare_grouped(KrylovSet& ks, const std::vector<size_t>& which, const JobMaker& make, bool fp64,
                            hipStream_t st, Arena* ar) {
    std::map<std::tuple<int, int, int, int>, std::vector<PassJob>> groups;
    for (size_t i : which) {
        const Inst& in = ks.inst[i];
        const int pr = (fp64 || in.p->prec == IBDL_PREC_FP64) ? 0 : 1;
        PassJob jb = make(i);
        const int om = jb.out.u ? (jb.out.out ? 2 : 1) : 0;
        groups[std::make_tuple(in.p->dim, in.p->n, pr, om)].push_back(jb);
    }
    GroupedPass gp;
    Arena& arena = ar ? *ar : *ks.arena;
    for (auto& kv : groups) {
        auto pp = prepare_pass(kv.second, fp64);
        pp->upload(arena, st);
        gp.parts.push_back(std::move(pp));
    }
    arena_flush(arena, st);
    return gp;
}

static std::vector<size_t> all_of(const KrylovSet& ks) {
    std::vector<size_t> w(ks.inst.size());
    for (size_t i = 0; i < w.size(); ++i) w[i] = i;
    return w;
}

// ------------------------------------------------------------------ solve task
SolveTask::SolveTask(KrylovSet& ks, SolveIO io, const ibdl_solve_opts& o, hipStream_t st, bool graphs)
    : ks_(ks), io_(std::move(io)), o_(o), st_(st) {
    m_ = o.restart;
    R_ = ks.R;
    IBDL_HIP_TRY(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
    // stage timing records events around each stage kernel: those iterations stay eager
    use_graph_ = graphs && graphs_enabled();
    for (const Inst& in : ks.inst)
        if (in.p->tm->enabled) use_graph_ = false;
}

SolveTask::~SolveTask() {
    // replays may still be in flight when the task ends early on an error; the set
    // keeps its graph for later solves
    if (graph_unmarked_) (void)hipStreamSynchronize(st_);
    if (ev_) (void)hipEventDestroy(ev_);
}

bool SolveTask::ready() {
    if (phase_ == DONE) return true;
    const hipError_t e = hipEventQuery(ev_);
    if (e == hipSuccess) return true;
    if (e == hipErrorNotReady) return false;
    (void)hipGetLastError();
    throw Error{IBDL_ERR_HIP, std::string("device work of a solve failed: ") + hipGetErrorString(e)};
}

void SolveTask::wait() {
    if (phase_ != DONE) IBDL_HIP_TRY(hipEventSynchronize(ev_));
}

void SolveTask::run_to_end() {
    while (!done()) {
        wait();
        advance();
    }
}

void SolveTask::mark() {
    IBDL_HIP_TRY(hipGetLastError());
    IBDL_HIP_TRY(hipEventRecord(ev_, st_));
    graph_unmarked_ = false;
}

// the grid solution of instance i can come out of its residual pass: asked for,
// and (Neumann) taken with V_b = the boundary data
bool SolveTask::grid_fusable(size_t i) const {
    if (i >= io_.u.size() || !io_.u[i]) return false;
    if (ks_.inst[i].p->form != IBDL_FORM_DOUBLE_LAYER) return false;
    if (ks_.inst[i].p->bc == IBDL_DIRICHLET) return true;
    return i < io_.vb.size() && io_.vb[i] == io_.data[i];
}

// r = b - A x for every instance (operator in FP64 when fp64, else the plans' precision).
// The FP64 residual of the system itself (b = the pool k.b) of an instance whose
// grid solution is asked for is formed from the boundary data: with
// u = L^-1 (g~ - S~ x [- S V_b]), Dirichlet r = U_b - x/2 - S* u, Neumann
// r = x/2 - S* u (the same r, since b = U_b - S* L^-1 g~, resp.
// S* L^-1 (S V_b - g~)); with_grid: u, the grid solution for the density x,
// is written by the same pass.
void SolveTask::residual(const double* b, const double* x, double* r, bool fp64, bool with_grid) {
    KWork& k = ks_.w;
    const bool system = fp64 && b == k.b;
    auto make = [&](size_t i) {
        // A x = -S* L^-1 S~ x + s x/2, so b - A x = S* L^-1 S~ x - s x/2 + b
        const Inst& in = ks_.inst[i];
        const size_t off = k.hxoff[in.r0];
        if (system && grid_fusable(i)) {
            PipeIn pi;
            pi.q_dip = x + off;
            pi.c_dip = -1.0;
            pi.pack_q = true;
            if (in.p->bc == IBDL_NEUMANN) {
                pi.q_mono = io_.data[i];
                pi.c_mono = -1.0;
            }
            pi.grid = io_.g[i];
            pi.c_grid = 1.0;
            PipeOut po;
            po.u = with_grid ? io_.u[i] : nullptr;
            po.out = r + off;
            po.cA = -1.0;
            po.in = x + off;
            if (in.p->bc == IBDL_DIRICHLET) {
                po.cB = -0.5;
                po.in2 = io_.data[i];
                po.cC = 1.0;
            } else {
                po.cB = 0.5;
            }
            if (with_grid) grid_done_[i] = 1;
            return PassJob{in.p, in.nrhs, pi, po};
        }
        PipeIn pi;
        pi.q_dip = x + off;
        pi.c_dip = 1.0;
        pi.pack_q = true;
        if (in.p->form == IBDL_FORM_COMPLETED) {
            // the completion's single layer: A x = -S* D0^-1 (S~ + eta S) x + x/2
            pi.q_mono = x + off;
            pi.c_mono = in.p->eta;
        }
        PipeOut po;
        po.out = r + off;
        po.cA = 1.0;
        po.in = x + off;
        po.cB = in.p->bc == IBDL_DIRICHLET ? -0.5 : 0.5;
        po.in2 = b + off;
        po.cC = 1.0;
        return PassJob{in.p, in.nrhs, pi, po};
    };
    prepare_grouped(ks_, all_of(ks_), make, fp64, st_).run(0, st_);
}

// per-rhs 2-norms of a pool into a host staging array (read after the next wait point)
void SolveTask::norms_async(const double* pool, double* host) {
    KWork& k = ks_.w;
    KArgs a = kargs(ks_, m_);
    hipLaunchKernelGGL(k_sumsq, dim3(k.nblk, R_), dim3(GT), 0, st_, a, pool);
    hipLaunchKernelGGL(k_norms, dim3((R_ + 63) / 64), dim3(64), 0, st_, a);
    IBDL_HIP_TRY(hipMemcpyAsync(host, k.nrm, R_ * sizeof(double), hipMemcpyDeviceToHost, st_));
}

void SolveTask::snapshot(int buf) {
    KWork& k = ks_.w;
    Staging hs = staging(k, R_);
    IBDL_HIP_TRY(hipMemcpyAsync(hs.resid[buf], k.resid, (size_t)R_ * (sizeof(double) + 4 * sizeof(int32_t)),
                                hipMemcpyDeviceToHost, st_));
}

// a private stream to record graphs on (recording launches nothing)
static hipStream_t capture_stream() {
    thread_local struct CS {
        hipStream_t s = nullptr;
        ~CS() {
            if (s) (void)hipStreamDestroy(s);
        }
    } cs;
    if (!cs.s) IBDL_HIP_TRY(hipStreamCreateWithFlags(&cs.s, hipStreamNonBlocking));
    return cs.s;
}

// Records 2^g Arnoldi steps (each: operator pass, both Gram-Schmidt passes) whose
// step indices are a base read from device memory plus 0, 1, ... 2^g - 1, and one
// increment of the base by 2^g; instantiates the graph or updates the set's
// executable graph of that length in place.  On failure: false, and the solve goes
// on without graphs.
bool SolveTask::capture_steps(int g) {
    KWork& k = ks_.w;
    KArgs a = kargs(ks_, m_);
    a.jp = k.jcur;
    const dim3 vg(k.nblk, R_);
    const int c = 1 << g;
    const hipStream_t cs = capture_stream();
    hipGraph_t graph = nullptr;
    IBDL_HIP_TRY(hipGetLastError());
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    capturing() = true;
    bool ok = true;
    try {
        for (int t = 0; t < c; ++t) {
            k.op->run_dev(k.jcur, t, cs);
            hipLaunchKernelGGL(k_orth, vg, dim3(GT), 0, cs, a, t);
            hipLaunchKernelGGL(k_orth_final, vg, dim3(GT), 0, cs, a, t);
        }
        hipLaunchKernelGGL(k_add_j, dim3(1), dim3(1), 0, cs, k.jcur, c);
    } catch (const Error&) {
        ok = false;
    }
    capturing() = false;
    if (hipStreamEndCapture(cs, &graph) != hipSuccess || !graph) ok = false;
    if (hipGetLastError() != hipSuccess) ok = false;
    hipGraphExec_t& ex = k.gexec[g];
    if (ok && ex) {
        // replays of the previous recording queued since the last wait point finish first
        if (graph_unmarked_) IBDL_HIP_TRY(hipStreamSynchronize(st_));
        hipGraphExecUpdateResult res;
        hipGraphNode_t bad = nullptr;
        if (hipGraphExecUpdate(ex, graph, &bad, &res) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(ex);
            ex = nullptr;
        }
    }
    if (ok && !ex && hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        ex = nullptr;
        ok = false;
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (ok) note_graphs(1, 0);
    return ok;
}

// c Arnoldi steps from step j0: with graphs, replays of 8, 4, 2 and 1 recorded
// steps (largest first), else every kernel launched on its own
void SolveTask::enqueue_iters(int j0, int c) {
    KWork& k = ks_.w;
    if (c <= 0) return;
    if (use_graph_ && k.op_ran && !k.graph_valid) {
        bool ok = true;
        for (int g = 0; g < KWork::kGraphLevels && ok; ++g) ok = capture_steps(g);
        k.graph_valid = ok;
        if (!ok) use_graph_ = false;
    }
    if (use_graph_ && k.graph_valid) {
        if (dev_j_ != j0) hipLaunchKernelGGL(k_set_j, dim3(1), dim3(1), 0, st_, k.jcur, j0);
        int left = c, replays = 0;
        for (int g = KWork::kGraphLevels - 1; g >= 0; --g)
            for (; left >= (1 << g); left -= 1 << g, ++replays) IBDL_HIP_TRY(hipGraphLaunch(k.gexec[g], st_));
        dev_j_ = j0 + c;
        graph_unmarked_ = true;
        note_graphs(0, replays);
        return;
    }
    KArgs a = kargs(ks_, m_);
    const dim3 vg(k.nblk, R_);
    for (int t = 0; t < c; ++t) {
        const int j = j0 + t;
        k.op->run(j, st_);
        hipLaunchKernelGGL(k_orth, vg, dim3(GT), 0, st_, a, j);
        hipLaunchKernelGGL(k_orth_final, vg, dim3(GT), 0, st_, a, j);
    }
    k.op_ran = true;
}

// c Arnoldi steps: the state is looked at before the last one, which keeps the
// device busy during the host's decision
void SolveTask::enqueue_chunk(int c) {
    const int c1 = c > 1 ? c - 1 : 1;
    enqueue_iters(kj_, c1);
    kj_ += c1;
    ktotal_ += c1;
    snap_buf_ ^= 1;
    snapshot(snap_buf_);
    mark();
    snap_iter_ = kj_;
    enqueue_iters(kj_, c - c1);
    kj_ += c - c1;
    ktotal_ += c - c1;
    queued_after_ = c - c1;
}

// The operator step of an Arnoldi iteration, prepared once per restart length and
// set of plan workspaces: the step index selects the basis vectors on the device.
void SolveTask::prepare_op() {
    KWork& k = ks_.w;
    KArgs a = kargs(ks_, m_);
    for (const Inst& in : ks_.inst) ensure_workspace(in.p, in.nrhs);
    std::vector<const void*> key{reinterpret_cast<const void*>((intptr_t)m_)};
    for (const Inst& in : ks_.inst) {
        key.push_back(in.p->ws.spec);
        key.push_back(in.p->ws.part);
    }
    if (k.op && key == k.op_key) return;
    auto make = [&](size_t i) {
        const Inst& in = ks_.inst[i];
        const int M = in.p->M;
        const size_t vb = k.hvoff[in.r0];
        const size_t vs = (size_t)(k.cap_m + 1) * M;
        PipeIn pi;
        pi.q_dip = k.V + vb;
        pi.c_dip = 1.0;
        pi.q_stride = vs;
        pi.q_jstride = M;
        pi.skip = k.state + 4 * in.r0;
        pi.pack_q = true;
        if (in.p->form == IBDL_FORM_COMPLETED) {
            pi.q_mono = k.V + vb;
            pi.c_mono = in.p->eta;
        }
        PipeOut po;
        po.out = k.V + vb + M;
        po.out_stride = vs;
        po.out_jstride = M;
        po.cA = -1.0;
        po.in = k.V + vb;
        po.in_stride = vs;
        po.in_jstride = M;
        po.cB = in.p->bc == IBDL_DIRICHLET ? 0.5 : -0.5;
        po.dots_V = k.V + vb;
        po.dots_vstride = vs;
        po.dots_nv = 1;
        po.dots = a.part + (size_t)in.r0 * a.pstride;
        po.dots_rhs = a.pstride;
        po.dots_stride = m_ + 2;
        return PassJob{in.p, in.nrhs, pi, po};
    };
    // the previous tables were uploaded for an earlier solve, whose work is complete
    arena_reset(k.op_arena);
    k.op = std::make_shared<GroupedPass>(prepare_grouped(ks_, all_of(ks_), make, false, st_, &k.op_arena));
    k.op_key = key;
    k.op_ran = k.graph_valid = false;
}

// Restarted GMRES on A x = b (pool vectors) with each plan's operator in its own
// precision, for every rhs not marked in skip_, to the tolerances tol_ (relative
// to ||b_r||) within at most budget_[r] Arnoldi steps each; x_zero: start from
// x = 0, else from the iterate in x.
void SolveTask::kstart(const double* b, double* x, bool x_zero) {
    KWork& k = ks_.w;
    KArgs a = kargs(ks_, m_);
    const dim3 vg(k.nblk, R_);
    Staging hs = staging(k, R_);
    kb_ = b;
    kx_ = x;
    kmaxit_ = 0;
    for (int r = 0; r < R_; ++r)
        if (!skip_[r]) kmaxit_ = std::max(kmaxit_, budget_[r]);
    ktotal_ = kj_ = 0;
    prev_iter_ = -1;
    if (x_zero) {
        // from x = 0 every rhs starts at relative residual 1, so the first chunk
        // decision of the run already has a rate of reduction to go by
        prev_.assign(R_, 1.0);
        prev_iter_ = 0;
    }
    for (int r = 0; r < R_; ++r) {
        hs.tol[r] = tol_[r];
        hs.skip[r] = skip_[r];
        hs.skip[R_ + r] = budget_[r];
    }
    IBDL_HIP_TRY(hipMemcpyAsync(k.tolv, hs.tol, R_ * sizeof(double), hipMemcpyHostToDevice, st_));
    IBDL_HIP_TRY(hipMemcpyAsync(k.skip, hs.skip, 2 * R_ * sizeof(int32_t), hipMemcpyHostToDevice, st_));
    hipLaunchKernelGGL(k_sumsq, vg, dim3(GT), 0, st_, a, b);
    hipLaunchKernelGGL(k_set_bnorm, dim3((R_ + 63) / 64), dim3(64), 0, st_, a);
    const double* r0 = b;
    if (x_zero) {
        hipLaunchKernelGGL(k_pool_op, vg, dim3(GT), 0, st_, a, 0, x, (const double*)nullptr);
    } else {
        residual(b, x, k.r, false);
        r0 = k.r;
    }
    hipLaunchKernelGGL(k_sumsq, vg, dim3(GT), 0, st_, a, r0);
    hipLaunchKernelGGL(k_init_cycle, vg, dim3(GT), 0, st_, a, r0);

    dev_j_ = 0;
    prepare_op();
    // rhs already converged at the start skip every step on the device
    enqueue_chunk(std::min({3, m_, kmaxit_}));
    phase_ = ITER;
}

// end of a Krylov run: x += V y, then what follows it without a host decision
// (the FP64 residual of a refinement, or the outputs), up to one wait point
void SolveTask::after_krylov() {
    KWork& k = ks_.w;
    KArgs a = kargs(ks_, m_);
    Staging hs = staging(k, R_);
    hipLaunchKernelGGL(k_backsolve, dim3(R_), dim3(BS_T), 0, st_, a);
    hipLaunchKernelGGL(k_update_x, dim3(k.nblk, R_), dim3(GT), 0, st_, a, kx_);
    hipLaunchKernelGGL(k_reset_j, dim3((R_ + 63) / 64), dim3(64), 0, st_, a);
    dev_j_ = 0;
    snap_buf_ ^= 1;
    snapshot(snap_buf_);
    if (refining_) hipLaunchKernelGGL(k_pool_op, dim3(k.nblk, R_), dim3(GT), 0, st_, a, 1, k.x, (const double*)k.d);
    if (any_mixed_) {
        // the grid solutions come with the residual of what may be the final iterate:
        // not with the one after the first FP32-operator solve when tol lies below
        // where that solve stops (its residual is then above tol; should it meet tol
        // after all, output() computes the grid solutions in a pass of their own)
        const bool maybe_final = refining_ || o_.tol >= kMixedFirstTol;
        residual(k.b, k.x, k.rr, true, maybe_final);
        norms_async(k.rr, hs.nrm);
    } else {
        if (o_.true_residual) {
            residual(k.b, k.x, k.rr, true);
            norms_async(k.rr, hs.nrm);
        }
        output();
    }
    mark();
    phase_ = KEND;
}

void SolveTask::collect() {
    Staging hs = staging(ks_.w, R_);
    const int32_t* state = hs.state[snap_buf_];
    const double* resid = hs.resid[snap_buf_];
    for (int r = 0; r < R_; ++r) {
        if (skip_[r]) continue;
        iters_[r] += state[4 * r + ST_ITERS];
        est_[r] = resid[r];
        int s = state[4 * r + ST_STATUS];
        if (s == IBDL_OK && !(resid[r] <= tol_[r])) s = IBDL_ERR_NOCONV;
        status_[r] = s;
    }
}

// outputs after a mixed solve: the FP64 residual of rhs that have none yet
// (when asked for), the solution copies and the grid solutions
void SolveTask::finish_mixed() {
    bool any = false;
    for (int r = 0; r < R_; ++r) any |= truer_[r] < 0.0;
    fill_true_ = o_.true_residual && any;
    if (fill_true_) {
        KWork& k = ks_.w;
        residual(k.b, k.x, k.rr, true);
        norms_async(k.rr, staging(k, R_).nrm);
    }
    output();
    mark();
    phase_ = OUT;
}

void SolveTask::output() {
    KWork& k = ks_.w;
    const size_t NI = ks_.inst.size();
    std::vector<size_t> grid;
    std::vector<CopyJob> copies;
    for (size_t i = 0; i < NI; ++i) {
        const Inst& in = ks_.inst[i];
        copies.push_back(CopyJob{io_.sol[i], k.x + k.hxoff[in.r0], (int64_t)in.nrhs * in.p->M});
        // grid solutions already written by the residual pass of the final iterate
        if (i < io_.u.size() && io_.u[i] && !grid_done_[i]) grid.push_back(i);
    }
    copy_multi(ks_, copies, st_);
    if (!grid.empty()) {
        // the grid solution (FP64): u = L^-1 (g~ - S~ Q) or L^-1 (g~ - S~ U_b - S V_b)
        auto make = [&](size_t i) {
            const Inst& in = ks_.inst[i];
            PipeIn pi;
            pi.q_dip = k.x + k.hxoff[in.r0];
            pi.c_dip = -1.0;
            pi.pack_q = true;
            if (in.p->bc == IBDL_NEUMANN) {
                pi.q_mono = io_.vb[i];
                pi.c_mono = -1.0;
            }
            pi.grid = io_.g[i];
            pi.c_grid = 1.0;
            PipeOut po;
            po.u = io_.u[i];
            return PassJob{in.p, in.nrhs, pi, po};
        };
        prepare_grouped(ks_, grid, make, true, st_).run(0, st_);
    }
}

void SolveTask::advance() {
    AllocStream as(st_);
    KWork& k = ks_.w;
    switch (phase_) {
    case BEGIN: {
        arena_reset(*ks_.arena);
        ensure_krylov(ks_, m_);
        const size_t NI = ks_.inst.size();
        grid_done_.assign(NI, 0);
        iters_.assign(R_, 0);
        status_.assign(R_, IBDL_OK);
        est_.assign(R_, 0.0);
        tol_.assign(R_, o_.tol);
        // mixed instances: the first FP32-operator solve stops near the FP32
        // operator's own accuracy; the FP64 refinement takes it to tol
        for (const Inst& in : ks_.inst)
            if (in.p->prec == IBDL_PREC_MIXED)
                for (int q = 0; q < in.nrhs; ++q) tol_[in.r0 + q] = std::max(o_.tol, kMixedFirstTol);
        skip_.assign(R_, 0);
        truer_.assign(R_, -1.0);
        fp64_.assign(R_, 0);
        any_mixed_ = false;
        for (const Inst& in : ks_.inst) any_mixed_ |= in.p->prec == IBDL_PREC_MIXED;
        refining_ = false;
        fill_true_ = false;
        round_ = 0;
        auto bytes_of = [&](const Inst& in) { return (size_t)in.nrhs * in.p->M * sizeof(double); };
        // right-hand sides in FP64 (Dirichlet: U_b - S* L^-1 g~; Neumann: S* L^-1 (S V_b - g~));
        // Dirichlet instances without forcing need no pass: b = U_b
        // Mixed instances whose grid solution is asked for form every FP64 residual
        // from the boundary data (see residual), so b only seeds their first
        // FP32-operator solve: it is formed in FP32 like that operator.
        std::vector<size_t> need64, need32;
        std::vector<CopyJob> copies;
        for (size_t i = 0; i < NI; ++i) {
            const Inst& in = ks_.inst[i];
            if (in.p->bc == IBDL_DIRICHLET && !io_.g[i])
                copies.push_back(CopyJob{k.b + k.hxoff[in.r0], io_.data[i], (int64_t)in.nrhs * in.p->M});
            else if (in.p->prec == IBDL_PREC_MIXED && grid_fusable(i))
                need32.push_back(i);
            else
                need64.push_back(i);
        }
        copy_multi(ks_, copies, st_);
        if (!need64.empty() || !need32.empty()) {
            auto make = [&](size_t i) {
                const Inst& in = ks_.inst[i];
                PipeIn pi;
                PipeOut po;
                po.out = k.b + k.hxoff[in.r0];
                if (in.p->bc == IBDL_DIRICHLET) {
                    pi.grid = io_.g[i];
                    pi.c_grid = 1.0;
                    po.cA = -1.0;
                    po.in = io_.data[i];
                    po.cB = 1.0;
                } else {
                    pi.q_mono = io_.data[i];
                    pi.c_mono = 1.0;
                    if (io_.g[i]) {
                        pi.grid = io_.g[i];
                        pi.c_grid = -1.0;
                    }
                    po.cA = 1.0;
                }
                return PassJob{in.p, in.nrhs, pi, po};
            };
            if (!need64.empty()) prepare_grouped(ks_, need64, make, true, st_).run(0, st_);
            if (!need32.empty()) prepare_grouped(ks_, need32, make, false, st_).run(0, st_);
        }
        bool any_x0 = false;
        for (size_t i = 0; i < io_.x0.size(); ++i) any_x0 |= io_.x0[i] != nullptr;
        if (any_x0) {
            for (size_t i = 0; i < NI; ++i) {
                const Inst& in = ks_.inst[i];
                double* dst = k.x + k.hxoff[in.r0];
                if (i < io_.x0.size() && io_.x0[i])
                    IBDL_HIP_TRY(hipMemcpyAsync(dst, io_.x0[i], bytes_of(in), hipMemcpyDeviceToDevice, st_));
                else
                    IBDL_HIP_TRY(hipMemsetAsync(dst, 0, bytes_of(in), st_));
            }
        }
        norms_async(k.b, staging(k, R_).bn);
        budget_.assign(R_, o_.maxit);
        kstart(k.b, k.x, !any_x0);
        return;
    }
    case ITER: {
        Staging hs = staging(k, R_);
        const int32_t* state = hs.state[snap_buf_];
        const double* resid = hs.resid[snap_buf_];
        bool all = true;
        for (int r = 0; r < R_ && all; ++r) all = state[4 * r + ST_DONE] != 0;
        if (all || ktotal_ >= kmaxit_) {
            after_krylov();
            return;
        }
        // steps still needed by the slowest rhs at its observed rate of residual
        // reduction, less those already queued behind the snapshot (1..8)
        int need = 3;
        if (prev_iter_ >= 0 && snap_iter_ > prev_iter_) {
            need = 1;
            const int d = snap_iter_ - prev_iter_;
            for (int r = 0; r < R_; ++r) {
                if (state[4 * r + ST_DONE]) continue;
                const double now = resid[r], before = prev_[r];
                int nr = 8;
                if (now > 0.0 && before > now) {
                    const double rate = std::pow(now / before, 1.0 / d);
                    if (rate < 1.0) nr = (int)std::ceil(std::log(tol_[r] / now) / std::log(rate));
                }
                need = std::max(need, std::min(std::max(nr, 1), 8));
            }
        }
        prev_.assign(resid, resid + R_);
        prev_iter_ = snap_iter_;
        const int want = need - queued_after_;
        if (want <= 0 && queued_after_ > 0 && kj_ < m_) {
            // the step queued behind the snapshot is expected to finish every rhs:
            // look at its state before queuing more (a further step would find every
            // rhs done and only cost its launches; a wrong guess costs one wait)
            snap_buf_ ^= 1;
            snapshot(snap_buf_);
            mark();
            snap_iter_ = kj_;
            queued_after_ = 0;
            return;
        }
        int c = std::max(1, std::min(8, want));
        if (kj_ >= m_) {
            // cycle end: restart the rhs still running from their current iterate
            KArgs a = kargs(ks_, m_);
            const dim3 vg(k.nblk, R_);
            hipLaunchKernelGGL(k_backsolve, dim3(R_), dim3(BS_T), 0, st_, a);
            hipLaunchKernelGGL(k_update_x, vg, dim3(GT), 0, st_, a, kx_);
            hipLaunchKernelGGL(k_reset_j, dim3((R_ + 63) / 64), dim3(64), 0, st_, a);
            dev_j_ = 0;
            residual(kb_, kx_, k.r, false);
            hipLaunchKernelGGL(k_sumsq, vg, dim3(GT), 0, st_, a, k.r);
            hipLaunchKernelGGL(k_init_cycle, vg, dim3(GT), 0, st_, a, k.r);
            kj_ = 0;
            prev_iter_ = -1;
            c = 3;
        }
        c = std::min({c, m_ - kj_, kmaxit_ - ktotal_});
        if (c <= 0) {
            after_krylov();
            return;
        }
        enqueue_chunk(c);
        return;
    }
    case KEND: {
        collect();
        Staging hs = staging(k, R_);
        bn_.assign(hs.bn, hs.bn + R_);
        if (!any_mixed_) {
            if (o_.true_residual)
                for (int r = 0; r < R_; ++r) {
                    truer_[r] = bn_[r] > 0.0 ? hs.nrm[r] / bn_[r] : 0.0;
                    fp64_[r] += 1;
                }
            phase_ = DONE;
            return;
        }
        if (!refining_) {
            // FP64 iterative refinement of the mixed instances: r = b - A x with
            // the FP64 operator, correct with the FP32-operator solve of A d = r, x += d
            for (const Inst& in : ks_.inst)
                if (in.p->prec != IBDL_PREC_MIXED)
                    for (int q = 0; q < in.nrhs; ++q) skip_[in.r0 + q] = 1;
            refining_ = true;
            round_ = 0;
        } else {
            ++round_;
        }
        bool all = true;
        for (int r = 0; r < R_; ++r) {
            if (skip_[r]) continue;
            fp64_[r] += 1;
            const double rn = hs.nrm[r];
            const double rel = bn_[r] > 0.0 ? rn / bn_[r] : 0.0;
            truer_[r] = rel;
            est_[r] = rel;
            if (!std::isfinite(rel)) {
                status_[r] = IBDL_ERR_NUMERIC;
                skip_[r] = 1;
            } else if (rel <= o_.tol || status_[r] == IBDL_ERR_NUMERIC) {
                if (status_[r] == IBDL_ERR_NOCONV) status_[r] = IBDL_OK;
                skip_[r] = 1;
            } else {
                all = false;
                // reduce the correction's residual to the target, no further than the FP32 floor
                tol_[r] = std::max(o_.tol * bn_[r] / rn, 1e-6);
            }
        }
        if (all) {
            finish_mixed();
            return;
        }
        // every rhs keeps its own budget: maxit less the steps it has taken itself, so
        // a right-hand side ends as it would in a solve of its own, whatever the others
        bool any = false;
        for (int r = 0; r < R_; ++r) {
            if (skip_[r]) continue;
            budget_[r] = o_.maxit - iters_[r];
            if (round_ >= 4 || budget_[r] <= 0) {
                if (status_[r] != IBDL_ERR_NUMERIC) status_[r] = IBDL_ERR_NOCONV;
                skip_[r] = 1;
            } else {
                any = true;
            }
        }
        if (!any) {
            finish_mixed();
            return;
        }
        kstart(k.rr, k.d, true);
        return;
    }
    case OUT: {
        if (fill_true_) {
            Staging hs = staging(k, R_);
            for (int r = 0; r < R_; ++r)
                if (truer_[r] < 0.0) {
                    truer_[r] = bn_[r] > 0.0 ? hs.nrm[r] / bn_[r] : 0.0;
                    fp64_[r] += 1;
                }
        }
        phase_ = DONE;
        return;
    }
    case DONE:
        return;
    }
}

int SolveTask::total_iters() const {
    int t = 0;
    for (int v : iters_) t += v;
    return t;
}

void SolveTask::results(ibdl_solve_info* info, int* overall) const {
    int worst = IBDL_OK;
    for (int r = 0; r < R_; ++r) {
        const int s = status_[r];
        if (info) {
            info[r].iters = iters_[r];
            info[r].rel_resid_est = est_[r];
            info[r].rel_resid_true = truer_[r];
            info[r].status = s;
            info[r].fp64_applies = fp64_[r];
        }
        if (s == IBDL_ERR_NUMERIC) worst = IBDL_ERR_NUMERIC;
        else if (s == IBDL_ERR_NOCONV && worst == IBDL_OK) worst = IBDL_ERR_NOCONV;
    }
    if (overall) *overall = worst;
}

void solve_set(KrylovSet& ks, const std::vector<const double*>& data, const std::vector<const double*>& g,
               const std::vector<const double*>& x0, const ibdl_solve_opts& o, const std::vector<double*>& sol,
               ibdl_solve_info* info, hipStream_t st, int* overall, const std::vector<double*>& u) {
    // nothing queued earlier reads argument tables any more once the stream is idle
    IBDL_HIP_TRY(hipStreamSynchronize(st));
    SolveIO io;
    io.data = data;
    io.g = g;
    io.x0 = x0;
    io.sol = sol;
    io.u = u;
    // Neumann grid solutions take V_b = the boundary data
    io.vb = data;
    SolveTask t(ks, std::move(io), o, st);
    t.run_to_end();
    t.results(info, overall);
}

}  // namespace ibdl
