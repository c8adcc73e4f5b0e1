// Plan construction: everything that depends only on the geometry and grid.
//
//  * cell binning: c_d = floor((X_d - lo_d)/h) mod n in IEEE FP64, key = row-major
//    cell index with x fastest; stable order of (key, caller index) as the order
//    of the 64-bit composites (key << 32 | index) -- unique, so the order of equal
//    cell keys is the caller order -- by ranking (small point counts) or a
//    bitonic sort;
//  * per point the 1-D delta taps phi(p - t) for p = c-1..c+2 (Sec. 5.2);
//  * the sparse dipole spread S~ q = div(S (q n)) (Sec. 5.2) and, for Neumann
//    plans, the monopole spread S (the discrete spread of Sec. 5.2),
//    as rows over the active grid nodes: entries per node are counted from the
//    points' stencils, and each node then collects its entries from the cells
//    around it and orders them by caller index -- no global sort of the entries;
//    every (node, point) pair the stencil reaches is one entry;
//  * the x-lines that receive forcing and the x-lines interpolated from;
//  * twiddles exp(-2 pi i m/n) and the symbol terms: (4/h^2) sin^2(pi m/n) for the
//    finite-difference Laplacian (Sec. 5.1), (2 pi k/L)^2 with k the signed
//    frequency for the Fourier-spectral one (Sec. 6.2.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <cmath>
#include <cstring>

#include "plan.h"

namespace ibdl {

// ------------------------------------------------------------------ alloc
static thread_local hipStream_t t_alloc_stream = nullptr;

hipStream_t alloc_stream() { return t_alloc_stream; }
AllocStream::AllocStream(hipStream_t s) : prev(t_alloc_stream) { t_alloc_stream = s; }
AllocStream::~AllocStream() { t_alloc_stream = prev; }

// the default pool of the current device keeps freed memory instead of returning it
static void keep_pool_memory() {
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(mu);
    if (std::find(done.begin(), done.end(), dev) != done.end()) return;
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    done.push_back(dev);
}

void* dev_alloc(std::vector<void*>& owner, size_t bytes) {
    keep_pool_memory();
    void* ptr = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMallocAsync(&ptr, bytes, t_alloc_stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{IBDL_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    owner.push_back(ptr);
    return ptr;
}

void dev_free(void* ptr) {
    if (ptr) (void)hipFreeAsync(ptr, t_alloc_stream);
}

static std::mutex g_pinned_mu;
static std::vector<std::pair<void*, size_t>> g_pinned_free;
static std::vector<std::pair<void*, size_t>> g_pinned_used;

void* pinned_get(size_t bytes) {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    size_t best = SIZE_MAX;
    int bi = -1;
    for (size_t i = 0; i < g_pinned_free.size(); ++i)
        if (g_pinned_free[i].second >= bytes && g_pinned_free[i].second < best) {
            best = g_pinned_free[i].second;
            bi = (int)i;
        }
    if (bi >= 0) {
        auto blk = g_pinned_free[bi];
        g_pinned_free.erase(g_pinned_free.begin() + bi);
        g_pinned_used.push_back(blk);
        return blk.first;
    }
    const size_t cap = std::max<size_t>((bytes + 4095) / 4096 * 4096, 4096);
    void* h = nullptr;
    if (hipHostMalloc(&h, cap) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{IBDL_ERR_OOM, "pinned host allocation failed"};
    }
    g_pinned_used.emplace_back(h, cap);
    return h;
}

void pinned_put(void* ptr) {
    if (!ptr) return;
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    for (size_t i = 0; i < g_pinned_used.size(); ++i)
        if (g_pinned_used[i].first == ptr) {
            g_pinned_free.push_back(g_pinned_used[i]);
            g_pinned_used.erase(g_pinned_used.begin() + i);
            return;
        }
}
void* dev_alloc(ibdl_plan p, size_t bytes) { return dev_alloc(p->allocs, bytes); }

template <typename T>
static T* alloc_n(ibdl_plan p, size_t n) {
    return reinterpret_cast<T*>(dev_alloc(p, n * sizeof(T)));
}
// construction temporaries, freed when the plan is built
template <typename T>
static T* tmp_n(ibdl_plan p, size_t n) {
    return reinterpret_cast<T*>(dev_alloc(p->build_tmp, n * sizeof(T)));
}

static inline int nblocks(size_t n, int t) { return (int)((n + t - 1) / t); }

// ------------------------------------------------------------------ kernels
__global__ void k_bin(const double* __restrict__ X, int M, int dim, int n, double lo0, double lo1,
                      double lo2, double h, uint32_t* key, int32_t* cell_c, double* frac,
                      int* bad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const double lo[3] = {lo0, lo1, lo2};
    uint32_t kk = 0, stride = 1;
    for (int d = 0; d < dim; ++d) {
        const double x = X[(size_t)k * dim + d];
        if (!isfinite(x)) bad[0] = 1;
        const double t = (x - lo[d]) / h;
        const double fl = floor(t);
        long long c = (long long)fl % n;
        if (c < 0) c += n;
        cell_c[3 * k + d] = (int32_t)c;
        frac[3 * k + d] = t - fl;
        kk += (uint32_t)c * stride;
        stride *= (uint32_t)n;
    }
    for (int d = dim; d < 3; ++d) { cell_c[3 * k + d] = 0; frac[3 * k + d] = 0.0; }
    key[k] = kk;
}

__global__ void k_check_geom(const double* __restrict__ nrm, const double* __restrict__ w, int M,
                             int dim, int* bad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    double s = 0;
    for (int d = 0; d < dim; ++d) {
        const double v = nrm[(size_t)k * dim + d];
        if (!isfinite(v)) bad[0] = 1;
        s += v * v;
    }
    if (!(fabs(s - 1.0) < 1e-6)) bad[1] = 1;
    if (!(w[k] > 0.0) || !isfinite(w[k])) bad[2] = 1;
}

__global__ void k_copy_geom(const double* __restrict__ X, const double* __restrict__ nrm,
                            const double* __restrict__ w, int M, int dim, double* X3, double* nrm3, double* w1) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    for (int d = 0; d < 3; ++d) X3[3 * k + d] = d < dim ? X[(size_t)k * dim + d] : 0.0;
    for (int d = 0; d < 3; ++d) nrm3[3 * k + d] = d < dim ? nrm[(size_t)k * dim + d] : 0.0;
    w1[k] = w[k];
}

__global__ void k_composite(const uint32_t* __restrict__ key, int M, size_t n2, uint64_t* out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    out[i] = i < (size_t)M ? (((uint64_t)key[i]) << 32) | (uint64_t)i : ~0ull;
}

// bitonic sort ------------------------------------------------------------
constexpr int BIT_T = 1024;              // threads of the LDS kernels
constexpr int BIT_BLOCK = 8192;          // elements held in LDS by one block (64 KiB)
constexpr int BIT_PER = BIT_BLOCK / 2 / BIT_T;  // compare-exchanges per thread and step

__device__ __forceinline__ void bit_cmpx(uint64_t* a, size_t lo, size_t hi, bool asc) {
    const uint64_t x = a[lo], y = a[hi];
    if ((x > y) == asc) { a[lo] = y; a[hi] = x; }
}

// the block's elements into LDS and back, BIT_BLOCK / BIT_T per thread
__device__ __forceinline__ void bit_load(uint64_t* s, const uint64_t* a, size_t base) {
#pragma unroll
    for (int u = 0; u < BIT_BLOCK / BIT_T; ++u) s[threadIdx.x + u * BIT_T] = a[base + threadIdx.x + u * BIT_T];
}
__device__ __forceinline__ void bit_store(const uint64_t* s, uint64_t* a, size_t base) {
#pragma unroll
    for (int u = 0; u < BIT_BLOCK / BIT_T; ++u) a[base + threadIdx.x + u * BIT_T] = s[threadIdx.x + u * BIT_T];
}
// one step (k, j) on the block's elements: pair t = lo | hi with lo's bit j clear
__device__ __forceinline__ void bit_step(uint64_t* s, size_t base, size_t k, int j, bool fixed_dir, bool asc_all) {
#pragma unroll
    for (int u = 0; u < BIT_PER; ++u) {
        const int t = threadIdx.x + u * BIT_T;
        const int lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int hi = lo | j;
        const bool asc = fixed_dir ? asc_all : (((base + lo) & k) == 0);
        const uint64_t x = s[lo], y = s[hi];
        if ((x > y) == asc) { s[lo] = y; s[hi] = x; }
    }
    __syncthreads();
}

// Steps with j < BIT_GROUP pair elements of one aligned group of BIT_GROUP: each
// thread holds the group 8t..8t+7 in registers for them (one LDS round trip and one
// barrier for up to three steps), stages k from kmin to kmax with steps j < 8 of each
constexpr int BIT_GROUP = BIT_BLOCK / BIT_T;  // 8
static_assert(BIT_GROUP == 8, "register steps assume groups of eight");
__device__ __forceinline__ void bit_group_steps(uint64_t* s, size_t base, int kmin, int kmax, bool fixed_dir,
                                                bool asc_all) {
    const int g0 = (int)threadIdx.x * BIT_GROUP;
    uint64_t v[BIT_GROUP];
#pragma unroll
    for (int i = 0; i < BIT_GROUP; ++i) v[i] = s[g0 + i];
    for (int k = kmin; k <= kmax; k <<= 1) {
#pragma unroll
        for (int j = 4; j > 0; j >>= 1) {
            if (j >= k) continue;  // stage k has steps j = k/2 .. 1
#pragma unroll
            for (int i = 0; i < BIT_GROUP; ++i) {
                if (i & j) continue;
                const bool asc = fixed_dir ? asc_all : (((base + g0 + i) & (size_t)k) == 0);
                if ((v[i] > v[i | j]) == asc) {
                    const uint64_t t = v[i];
                    v[i] = v[i | j];
                    v[i | j] = t;
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < BIT_GROUP; ++i) s[g0 + i] = v[i];
    __syncthreads();
}

// all stages with k <= BIT_BLOCK inside each block
__global__ __launch_bounds__(BIT_T) void k_bitonic_local_sort(uint64_t* a) {
    __shared__ uint64_t s[BIT_BLOCK];
    const size_t base = (size_t)blockIdx.x * BIT_BLOCK;
    bit_load(s, a, base);
    __syncthreads();
    bit_group_steps(s, base, 2, BIT_GROUP, false, true);  // stages k = 2, 4, 8 entirely
    for (int k = 2 * BIT_GROUP; k <= BIT_BLOCK; k <<= 1) {
        for (int j = k >> 1; j >= BIT_GROUP; j >>= 1) bit_step(s, base, (size_t)k, j, false, true);
        bit_group_steps(s, base, k, k, false, true);
    }
    bit_store(s, a, base);
}

// stages j < BIT_BLOCK of a merge with k > BIT_BLOCK
__global__ __launch_bounds__(BIT_T) void k_bitonic_local_merge(uint64_t* a, size_t k) {
    __shared__ uint64_t s[BIT_BLOCK];
    const size_t base = (size_t)blockIdx.x * BIT_BLOCK;
    bit_load(s, a, base);
    __syncthreads();
    const bool asc = ((base & k) == 0);
    for (int j = BIT_BLOCK >> 1; j >= BIT_GROUP; j >>= 1) bit_step(s, base, k, j, true, asc);
    // the group steps only need j < 8 (any stage value >= 8 gives all three)
    bit_group_steps(s, base, 2 * BIT_GROUP, 2 * BIT_GROUP, true, asc);
    bit_store(s, a, base);
}

__global__ void k_bitonic_global(uint64_t* a, size_t npairs, size_t k, size_t j) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npairs) return;
    const size_t lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
    const size_t hi = lo | j;
    bit_cmpx(a, lo, hi, (lo & k) == 0);
}

// steps j and j/2 of stage k together (j/2 >= BIT_BLOCK): thread t owns the four
// elements i0 | {0, h, j, j + h} (h = j/2, i0 with bits j and h clear), all in the
// same direction (k > j), and does step j's two compare-exchanges and then step
// j/2's two on them: half the passes over the array
__global__ void k_bitonic_global2(uint64_t* a, size_t nquads, size_t k, size_t j) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nquads) return;
    const size_t h = j >> 1;
    const size_t i0 = ((t & ~(h - 1)) << 2) | (t & (h - 1));
    const bool asc = (i0 & k) == 0;
    uint64_t v0 = a[i0], v1 = a[i0 | h], v2 = a[i0 | j], v3 = a[i0 | j | h];
    auto cx = [asc](uint64_t& x, uint64_t& y) {
        if ((x > y) == asc) {
            const uint64_t tmp = x;
            x = y;
            y = tmp;
        }
    };
    cx(v0, v2);
    cx(v1, v3);
    cx(v0, v1);
    cx(v2, v3);
    a[i0] = v0;
    a[i0 | h] = v1;
    a[i0 | j] = v2;
    a[i0 | j | h] = v3;
}

static size_t pow2_at_least(size_t n, size_t minv) {
    size_t p = minv;
    while (p < n) p <<= 1;
    return p;
}

// sorts a[0..n2) ascending; n2 a power of two >= BIT_BLOCK
static void bitonic_sort(uint64_t* a, size_t n2, hipStream_t st) {
    const int nb = (int)(n2 / BIT_BLOCK);
    hipLaunchKernelGGL(k_bitonic_local_sort, dim3(nb), dim3(BIT_T), 0, st, a);
    for (size_t k = 2 * BIT_BLOCK; k <= n2; k <<= 1) {
        size_t j = k >> 1;
        for (; j >= 2 * (size_t)BIT_BLOCK; j >>= 2)
            hipLaunchKernelGGL(k_bitonic_global2, dim3(nblocks(n2 / 4, 256)), dim3(256), 0, st, a,
                               n2 / 4, k, j);
        if (j >= (size_t)BIT_BLOCK)
            hipLaunchKernelGGL(k_bitonic_global, dim3(nblocks(n2 / 2, 256)), dim3(256), 0, st, a,
                               n2 / 2, k, j);
        hipLaunchKernelGGL(k_bitonic_local_merge, dim3(nb), dim3(BIT_T), 0, st, a, k);
    }
    IBDL_HIP_TRY(hipGetLastError());
}

// exclusive scan of int32 ----------------------------------------------------
constexpr int SCAN_T = 256, SCAN_PER = 8, SCAN_TILE = SCAN_T * SCAN_PER;

__global__ __launch_bounds__(SCAN_T) void k_scan_tile(const int32_t* in, int32_t* out, size_t n,
                                                      int32_t* sums) {
    __shared__ int32_t s[SCAN_T];
    const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_PER;
    int32_t v[SCAN_PER];
    int32_t tot = 0;
    for (int i = 0; i < SCAN_PER; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        tot += v[i];
    }
    s[threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int32_t add = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = s[threadIdx.x] - tot;
    for (int i = 0; i < SCAN_PER; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == SCAN_T - 1 && sums) sums[blockIdx.x] = s[SCAN_T - 1];
}

__global__ void k_scan_add(int32_t* out, size_t n, const int32_t* offs) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += offs[i / SCAN_TILE];
}

// out = exclusive scan of in (n entries; in place allowed: a tile reads its entries
// before it writes them); the total is out[n-1] plus in[n-1]
static void scan_excl(ibdl_plan p, const int32_t* in, int32_t* out, size_t n, hipStream_t st) {
    const size_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nt <= 1) {
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(SCAN_T), 0, st, in, out, n, (int32_t*)nullptr);
        return;
    }
    int32_t* sums = tmp_n<int32_t>(p, nt);
    int32_t* soff = tmp_n<int32_t>(p, nt);
    hipLaunchKernelGGL(k_scan_tile, dim3((int)nt), dim3(SCAN_T), 0, st, in, out, n, sums);
    scan_excl(p, sums, soff, nt, st);
    hipLaunchKernelGGL(k_scan_add, dim3(nblocks(n, 256)), dim3(256), 0, st, out, n, soff);
}

// ------------------------------------------------------------------ sorted geometry
// Rank sort for small point counts: the sorted position of point k is the number of
// composites (key << 32 | index) below its own -- all distinct, so the ranks are a
// permutation and equal keys keep the caller order.  A block ranks RS_K points,
// RS_SPLIT threads per point each counting over a quarter of every tile of RS_T.
constexpr int RS_K = 64, RS_SPLIT = 4, RS_T = RS_K * RS_SPLIT;
#ifndef IBDL_RANK_SORT_MAX
#define IBDL_RANK_SORT_MAX 16384
#endif
constexpr int RANK_SORT_MAX = IBDL_RANK_SORT_MAX;  // above this the bitonic sort is faster

__global__ __launch_bounds__(RS_T) void k_rank_sort(const uint32_t* __restrict__ key, int M, uint32_t* perm,
                                                    uint32_t* skey, uint32_t* invperm) {
    __shared__ uint64_t tile[RS_T];
    __shared__ int part[RS_SPLIT][RS_K];
    const int kk = threadIdx.x % RS_K, q = threadIdx.x / RS_K;
    const int k = blockIdx.x * RS_K + kk;
    const uint64_t mine = k < M ? (((uint64_t)key[k]) << 32) | (uint64_t)k : ~0ull;
    int rank = 0;
    for (int base = 0; base < M; base += RS_T) {
        const int j = base + threadIdx.x;
        tile[threadIdx.x] = j < M ? (((uint64_t)key[j]) << 32) | (uint64_t)j : ~0ull;
        __syncthreads();
#pragma unroll 16
        for (int t = 0; t < RS_K; ++t) rank += tile[q * RS_K + t] < mine;
        __syncthreads();
    }
    part[q][kk] = rank;
    __syncthreads();
    if (q == 0 && k < M) {
        int r = 0;
        for (int i = 0; i < RS_SPLIT; ++i) r += part[i][kk];
        perm[r] = (uint32_t)k;
        skey[r] = key[k];
        invperm[k] = (uint32_t)r;
    }
}

__global__ void k_unpack(const uint64_t* __restrict__ srt, int M, uint32_t* perm, uint32_t* skey,
                         uint32_t* invperm) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= M) return;
    const uint64_t v = srt[s];
    const uint32_t k = (uint32_t)(v & 0xffffffffull);
    perm[s] = k;
    skey[s] = (uint32_t)(v >> 32);
    invperm[k] = (uint32_t)s;
}

__global__ void k_taps(const uint32_t* __restrict__ perm, const int32_t* __restrict__ cell_c,
                       const double* __restrict__ frac, int M, int dim, int kind,
                       int32_t* cell_s, double* taps64, float* taps32) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= M) return;
    const uint32_t k = perm[s];
    for (int d = 0; d < 3; ++d) {
        cell_s[3 * s + d] = cell_c[3 * k + d];
        for (int i = 0; i < 4; ++i) {
            double v = 0.0;
            if (d < dim) {
                // node p = c - 1 + i, p - t = i - 1 - frac
                const double r = (double)(i - 1) - frac[3 * k + d];
                v = kind == IBDL_DELTA_PESKIN4 ? phi_peskin4(r) : phi_cosine4(r);
            }
            taps64[12 * s + 4 * d + i] = v;
            taps32[12 * s + 4 * d + i] = (float)v;
        }
    }
}

// first sorted position whose key / n >= line, for line in [0, nlines]
__global__ void k_line_start(const uint32_t* __restrict__ skey, int M, int n, int nlines,
                             int32_t* ls) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > nlines) return;
    int lo = 0, hi = M;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)(skey[mid] / (uint32_t)n) < l) lo = mid + 1; else hi = mid;
    }
    ls[l] = lo;
}

// ------------------------------------------------------------------ spread matrices
// A point in cell c reaches the nodes c + r with r in -2..3 per axis and at most one
// axis outside -1..2 (the dipole: the centred difference reaches one node further
// along its own axis; at the other nodes of the 6^d box every term vanishes), or r
// in -1..2 per axis (the monopole).  Seen from a node line (y, z): the points of the
// x-lines (y - ry, z - rz) reach it, those of a line with ry or rz outside -1..2 at
// x-offsets -1..2 only, the others at lo..hi.

// A_d(r) = phi(c - 1 + i - t) at r = i - 1 in -1..2, zero outside
__device__ __forceinline__ double tap_at(const double* t4, int r) {
    return (r >= -1 && r <= 2) ? t4[r + 1] : 0.0;
}

// weight of point k (sorted position s, stencil offsets r) at a node: the dipole
// (w_k / h^d) sum_d n_d (A_d(r_d+1) - A_d(r_d-1)) / (2h) prod_{e != d} A_e(r_e),
// or the monopole (w_k / h^d) prod_d A_d(r_d)
__device__ double entry_weight(const double* __restrict__ t, const double* __restrict__ nrm3, double wk, uint32_t k,
                               const int* r, int dim, double h, int dipole) {
    double hd = 1.0;
    for (int d = 0; d < dim; ++d) hd *= h;
    if (dipole) {
        double acc = 0.0;
        for (int d = 0; d < dim; ++d) {
            double term = (tap_at(t + 4 * d, r[d] + 1) - tap_at(t + 4 * d, r[d] - 1)) / (2.0 * h);
            for (int q = 0; q < dim; ++q)
                if (q != d) term *= tap_at(t + 4 * q, r[q]);
            acc += nrm3[3 * k + d] * term;
        }
        return wk / hd * acc;
    }
    double prod = 1.0;
    for (int d = 0; d < dim; ++d) prod *= tap_at(t + 4 * d, r[d]);
    return wk / hd * prod;
}

constexpr int CL_W = 2;  // node lines per block, one wavefront each

// f(s, x) for every (point, node) entry of node line l: s the point's sorted
// position, x the node's column; the lanes of the wavefront split each point line
template <typename F>
__device__ __forceinline__ void line_entries(int l, int dim, int n, int dipole, const int32_t* __restrict__ line_start,
                                             const uint32_t* __restrict__ skey, int lane, F&& f) {
    const int y = l % n, z = l / n;
    const int lo = dipole ? -2 : -1, hi = dipole ? 3 : 2;
    const int zlo = dim == 3 ? lo : 0, zhi = dim == 3 ? hi : 0;
    for (int rz = zlo; rz <= zhi; ++rz) {
        int cz = z - rz;
        cz += cz < 0 ? n : 0;
        cz -= cz >= n ? n : 0;
        for (int ry = lo; ry <= hi; ++ry) {
            const int outside = (ry < -1 || ry > 2) + (rz < -1 || rz > 2);
            if (outside > 1) continue;
            const int xlo = outside ? -1 : lo, xhi = outside ? 2 : hi;
            int cy = y - ry;
            cy += cy < 0 ? n : 0;
            cy -= cy >= n ? n : 0;
            const int pl = cz * n + cy;
            const int s1 = line_start[pl + 1];
            for (int s = line_start[pl] + lane; s < s1; s += 64) {
                const int cx = (int)(skey[s] % (uint32_t)n);
                for (int rx = xlo; rx <= xhi; ++rx) {
                    // n >= 8: one periodic wrap at most
                    int x = cx + rx;
                    x += x < 0 ? n : 0;
                    x -= x >= n ? n : 0;
                    f(s, x);
                }
            }
        }
    }
}

// One wavefront per node line (lines l >= nlines only take part in the barriers):
// the entry count of every node of the line is summed in LDS (integer atomics:
// exact in any order) from the points of the x-lines around it.  PASS 1 writes the
// line's active-node and entry counts (line nlines: 0, so exclusive scans of
// nlines + 1 entries end in the totals).  PASS 2 takes those scans (the first active
// node and first entry of each line) and writes the line's active nodes in
// ascending column with their entry offsets, then places each entry's caller index
// and active index in its node's range through an LDS cursor; the order inside a
// node is settled by k_entry_order.  LDS: 2 n ints per wavefront.
template <int PASS>
__global__ __launch_bounds__(64 * CL_W) void k_csr_lines(int nlines, int dim, int n, int dipole,
                                                         const int32_t* __restrict__ line_start,
                                                         const uint32_t* __restrict__ skey,
                                                         const uint32_t* __restrict__ perm, int32_t* line_nact,
                                                         int32_t* line_nnz, const int32_t* __restrict__ act_off,
                                                         const int32_t* __restrict__ nnz_off, uint32_t* act_node,
                                                         int32_t* act_ptr, uint32_t* ent_k, int32_t* ent_a) {
    extern __shared__ int32_t lds_cl[];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int l = blockIdx.x * CL_W + w;
    const bool live = l < nlines;
    int32_t* cnt = lds_cl + (size_t)w * 2 * n;  // counts, then cursors
    int32_t* aid = cnt + n;                      // active index of each column (PASS 2)
    for (int x = lane; x < n; x += 64) cnt[x] = 0;
    __syncthreads();
    if (live) line_entries(l, dim, n, dipole, line_start, skey, lane, [&](int, int x) { atomicAdd(&cnt[x], 1); });
    __syncthreads();
    if (PASS == 1) {
        int na = 0, ne = 0;
        for (int x = lane; x < n; x += 64) {
            const int c = cnt[x];
            na += c > 0;
            ne += c;
        }
        for (int off = 32; off > 0; off >>= 1) {
            na += __shfl_xor(na, off, 64);
            ne += __shfl_xor(ne, off, 64);
        }
        if (lane == 0 && l <= nlines) {
            line_nact[l] = live ? na : 0;
            line_nnz[l] = live ? ne : 0;
        }
        return;
    }
    // columns [x0, x0 + C) per lane, in order; exclusive scans over the lanes
    const int C = (n + 63) / 64, x0 = lane * C, x1 = x0 + C < n ? x0 + C : n;
    int na = 0, ne = 0;
    for (int x = x0; x < x1; ++x) {
        const int c = cnt[x];
        na += c > 0;
        ne += c;
    }
    int pa = na, pe = ne;  // inclusive, then exclusive
    for (int off = 1; off < 64; off <<= 1) {
        const int ta = __shfl_up(pa, off, 64), te = __shfl_up(pe, off, 64);
        if (lane >= off) {
            pa += ta;
            pe += te;
        }
    }
    pa -= na;
    pe -= ne;
    if (live) {
        int a = act_off[l] + pa, e = nnz_off[l] + pe;
        for (int x = x0; x < x1; ++x) {
            const int c = cnt[x];
            if (c == 0) continue;
            act_node[a] = (uint32_t)l * (uint32_t)n + (uint32_t)x;
            act_ptr[a] = e;
            aid[x] = a;
            cnt[x] = e;
            ++a;
            e += c;
        }
    }
    __syncthreads();
    if (live)
        line_entries(l, dim, n, dipole, line_start, skey, lane, [&](int s, int x) {
            const int slot = atomicAdd(&cnt[x], 1);
            ent_k[slot] = perm[s];
            ent_a[slot] = aid[x];
        });
}

// Caller order within each node, one entry per thread: the entry's rank among its
// node's entries (caller indices are distinct) is its place -- the summation order
// of the spread.  K receives the ordered caller indices.
__global__ void k_entry_order(size_t nnz, const uint32_t* __restrict__ ent_k, const int32_t* __restrict__ ent_a,
                              const int32_t* __restrict__ act_ptr, uint32_t* K) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int a = ent_a[e];
    const int e0 = act_ptr[a], e1 = act_ptr[a + 1];
    const uint32_t v = ent_k[e];
    int rank = 0;
    for (int i = e0; i < e1; ++i) rank += ent_k[i] < v;
    K[e0 + rank] = v;
}

// entry weights and sorted positions, one entry per thread (K: the entries' caller
// indices, ent_a: their nodes' active indices)
__global__ void k_entry_weights(size_t nnz, const int32_t* __restrict__ ent_a,
                                const uint32_t* __restrict__ act_node, int dim, int n,
                                const int32_t* __restrict__ cell_s, const uint32_t* __restrict__ invperm,
                                const double* __restrict__ taps64, const double* __restrict__ nrm3,
                                const double* __restrict__ w1, double h, int dipole, const uint32_t* __restrict__ K,
                                uint32_t* S, double* W64, float* W32) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const uint32_t k = K[e];
    const uint32_t s = invperm[k];
    uint32_t rem = act_node[ent_a[e]];
    int r[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        const int p = (int)(rem % (uint32_t)n);
        rem /= (uint32_t)n;
        r[d] = ((p - cell_s[3 * s + d] + 2 + 2 * n) % n) - 2;   // in -2..3
    }
    const double wv = entry_weight(taps64 + 12 * (size_t)s, nrm3, w1[k], k, r, dim, h, dipole);
    S[e] = s;
    W64[e] = wv;
    W32[e] = (float)wv;
}

__global__ void k_set_i32(int32_t* p, int32_t v) { *p = v; }

// ------------------------------------------------------------------ line sets
__global__ void k_spread_mask(const int32_t* __restrict__ la, int nlines, uint8_t* mask,
                              int32_t* flag) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlines) return;
    const int v = la[l + 1] > la[l];
    mask[l] = (uint8_t)v;
    flag[l] = v;
}

// every x-line (cy-1..cy+2, cz-1..cz+2) a point interpolates from
__global__ void k_gather_mark(const int32_t* __restrict__ cell_s, int M, int dim, int n,
                              uint8_t* mask) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = dim == 3 ? 16 : 4;
    if (id >= M * per) return;
    const int s = id / per, j = id % per;
    const int cy = (cell_s[3 * s + 1] - 1 + (j % 4) + n) % n;
    const int cz = dim == 3 ? (cell_s[3 * s + 2] - 1 + j / 4 + n) % n : 0;
    mask[cz * n + cy] = 1;  // all writers store the same value
}

__global__ void k_mask_to_flag(const uint8_t* __restrict__ mask, int n, int32_t* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = mask[i];
}

__global__ void k_plane_mask(const uint8_t* __restrict__ lmask, int n, uint8_t* pmask,
                             int32_t* flag) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= n) return;
    int any = 0;
    for (int y = 0; y < n; ++y) any |= lmask[z * n + y];
    pmask[z] = (uint8_t)any;
    flag[z] = any;
}

__global__ void k_compact_list(const int32_t* __restrict__ flag, const int32_t* __restrict__ idx,
                               int n, int32_t* list) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) list[idx[i]] = i;
}

// ------------------------------------------------------------------ tables
__global__ void k_tables(int n, double h, double length, int spectral, double* tw64, float* tw32, double* s264,
                         float* s232) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double sv, cv;
    sincospi(2.0 * (double)m / (double)n, &sv, &cv);
    tw64[2 * m] = cv;
    tw64[2 * m + 1] = -sv;
    tw32[2 * m] = (float)cv;
    tw32[2 * m + 1] = (float)(-sv);
    double v;
    if (spectral) {
        const double k = 2.0 * M_PI * (double)(m <= n / 2 ? m : m - n) / length;
        v = k * k;
    } else {
        const double sp = sinpi((double)m / (double)n);
        v = 4.0 / (h * h) * sp * sp;
    }
    s264[m] = v;
    s232[m] = (float)v;
}

// 2-D inverse symbol in FP32, from FP64 terms: norm / lambda(kx, ky) with
// lambda = -(s2[kx] + s2[ky]) - alpha, 0 where lambda = 0 (the mean of a Poisson
// solve) and in the padding columns kx >= W of the last tile; layout [tile][ky][C]
__global__ void k_symtab(int n, int C, int W, size_t total, const double* __restrict__ s2, double alpha,
                         double norm, float* out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const size_t tile = (size_t)n * C;
    const int t = (int)(e / tile);
    const int rem = (int)(e - (size_t)t * tile);
    const int ky = rem / C, kx = t * C + rem % C;
    float v = 0.0f;
    if (kx < W) {
        const double lam = s2[ky] + (s2[kx] + alpha);
        if (lam != 0.0) v = (float)(-norm / lam);
    }
    out[e] = v;
}

// ------------------------------------------------------------------ host
// device counts gathered for one copy to the host
struct CountPtrs {
    const int32_t* p[8];
    int n;
};
__global__ void k_gather_counts(CountPtrs c, int32_t* out) {
    const int i = threadIdx.x;
    if (i < c.n) out[i] = *c.p[i];
}

// Flags (n entries and a zero at n) and their exclusive scan, whose entry n is the
// count; the list of set indices is written once the count is known.
struct Compaction {
    const int32_t* flag = nullptr;
    int32_t* idx = nullptr;
    int n = 0;
};
static Compaction flag_scan(ibdl_plan p, const int32_t* flag, int n, hipStream_t st) {
    Compaction c;
    c.flag = flag;
    c.n = n;
    c.idx = tmp_n<int32_t>(p, (size_t)n + 1);
    scan_excl(p, flag, c.idx, (size_t)n + 1, st);
    return c;
}
static int32_t* compact_list(ibdl_plan p, const Compaction& c, int cnt, hipStream_t st) {
    int32_t* list = alloc_n<int32_t>(p, (size_t)std::max(cnt, 1));
    hipLaunchKernelGGL(k_compact_list, dim3(nblocks(c.n, 256)), dim3(256), 0, st, c.flag, c.idx, c.n, list);
    return list;
}

static int entries_per_point(int dim, bool dipole) { return dipole ? (dim == 2 ? 32 : 160) : (dim == 2 ? 16 : 64); }

// First pass of a spread matrix: active nodes and entries per node line, scanned
// (c.line_act: the first active node of each line; the returned array: the first
// entry of each line); both scans end in the totals at index nlines.
static int32_t* csr_count(ibdl_plan p, Csr& c, bool dipole, hipStream_t st) {
    const int nl = p->nlines, n = p->n;
    if ((size_t)p->M * entries_per_point(p->dim, dipole) * sizeof(double) >= (size_t)INT32_MAX)
        throw Error{IBDL_ERR_ARG, "too many spread entries"};
    int32_t* ln = tmp_n<int32_t>(p, (size_t)nl + 1);
    int32_t* le = tmp_n<int32_t>(p, (size_t)nl + 1);
    const size_t lds = (size_t)CL_W * 2 * n * sizeof(int32_t);
    hipLaunchKernelGGL(k_csr_lines<1>, dim3(nblocks((size_t)nl + 1, CL_W)), dim3(64 * CL_W), lds, st, nl, p->dim, n,
                       dipole ? 1 : 0, p->line_start, p->skey, p->perm, ln, le, (const int32_t*)nullptr,
                       (const int32_t*)nullptr, (uint32_t*)nullptr, (int32_t*)nullptr, (uint32_t*)nullptr,
                       (int32_t*)nullptr);
    c.line_act = alloc_n<int32_t>(p, (size_t)nl + 1);
    scan_excl(p, ln, c.line_act, (size_t)nl + 1, st);
    int32_t* nnz_off = tmp_n<int32_t>(p, (size_t)nl + 1);
    scan_excl(p, le, nnz_off, (size_t)nl + 1, st);
    return nnz_off;
}

// Second pass: the active nodes, their entry offsets and the entries (caller order
// within a node, weights).  Every (point, stencil node) pair is one entry, so the
// counted total must be M times the stencil size.
static void csr_fill(ibdl_plan p, Csr& c, bool dipole, const int32_t* nnz_off, int nact, int nnz, hipStream_t st) {
    const int nl = p->nlines, n = p->n;
    if ((int64_t)nnz != (int64_t)p->M * entries_per_point(p->dim, dipole) || nact < 1)
        throw Error{IBDL_ERR_STATE, "internal: spread matrix entry count mismatch"};
    c.nact = nact;
    c.nnz = nnz;
    c.act_node = alloc_n<uint32_t>(p, (size_t)nact);
    c.act_ptr = alloc_n<int32_t>(p, (size_t)nact + 1);
    c.k = alloc_n<uint32_t>(p, (size_t)nnz);
    c.s = alloc_n<uint32_t>(p, (size_t)nnz);
    c.w64 = alloc_n<double>(p, (size_t)nnz);
    c.w32 = alloc_n<float>(p, (size_t)nnz);
    uint32_t* ent_k = tmp_n<uint32_t>(p, (size_t)nnz);
    int32_t* ent_a = tmp_n<int32_t>(p, (size_t)nnz);
    const size_t lds = (size_t)CL_W * 2 * n * sizeof(int32_t);
    hipLaunchKernelGGL(k_csr_lines<2>, dim3(nblocks(nl, CL_W)), dim3(64 * CL_W), lds, st, nl, p->dim, n,
                       dipole ? 1 : 0, p->line_start, p->skey, p->perm, (int32_t*)nullptr, (int32_t*)nullptr,
                       (const int32_t*)c.line_act, nnz_off, c.act_node, c.act_ptr, ent_k, ent_a);
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, st, c.act_ptr + nact, (int32_t)nnz);
    hipLaunchKernelGGL(k_entry_order, dim3(nblocks(nnz, 256)), dim3(256), 0, st, (size_t)nnz, ent_k, ent_a,
                       c.act_ptr, c.k);
    hipLaunchKernelGGL(k_entry_weights, dim3(nblocks(nnz, 256)), dim3(256), 0, st, (size_t)nnz, ent_a, c.act_node,
                       p->dim, n, p->cell, p->invperm, p->taps64, p->nrm, p->wgt, p->h, dipole ? 1 : 0, c.k, c.s,
                       c.w64, c.w32);
    IBDL_HIP_TRY(hipGetLastError());
}

void build_plan(ibdl_plan p, const ibdl_desc* d, hipStream_t st) {
    const int dim = p->dim, n = p->n, M = p->M;
    int32_t* bad = tmp_n<int32_t>(p, 4);
    IBDL_HIP_TRY(hipMemsetAsync(bad, 0, 4 * sizeof(int32_t), st));
    p->key = alloc_n<uint32_t>(p, M);
    int32_t* cell_c = tmp_n<int32_t>(p, 3 * (size_t)M);
    double* frac = tmp_n<double>(p, 3 * (size_t)M);
    hipLaunchKernelGGL(k_bin, dim3(nblocks(M, 256)), dim3(256), 0, st, d->X, M, dim, n, p->lo[0],
                       p->lo[1], p->lo[2], p->h, p->key, cell_c, frac, bad);
    hipLaunchKernelGGL(k_check_geom, dim3(nblocks(M, 256)), dim3(256), 0, st, d->normal, d->weight, M,
                       dim, bad);
    int32_t hb[4];
    IBDL_HIP_TRY(hipMemcpyAsync(hb, bad, sizeof(hb), hipMemcpyDeviceToHost, st));
    IBDL_HIP_TRY(hipStreamSynchronize(st));
    if (hb[0]) throw Error{IBDL_ERR_NUMERIC, "non-finite point coordinate or normal"};
    if (hb[1]) throw Error{IBDL_ERR_ARG, "normals must have unit length"};
    if (hb[2]) throw Error{IBDL_ERR_ARG, "weights must be positive and finite"};

    p->X = alloc_n<double>(p, 3 * (size_t)M);
    p->nrm = alloc_n<double>(p, 3 * (size_t)M);
    p->wgt = alloc_n<double>(p, M);
    hipLaunchKernelGGL(k_copy_geom, dim3(nblocks(M, 256)), dim3(256), 0, st, d->X, d->normal, d->weight, M,
                       dim, p->X, p->nrm, p->wgt);

    // stable order of (key, index)
    p->perm = alloc_n<uint32_t>(p, M);
    p->skey = alloc_n<uint32_t>(p, M);
    p->invperm = alloc_n<uint32_t>(p, M);
    if (M <= RANK_SORT_MAX) {
        hipLaunchKernelGGL(k_rank_sort, dim3(nblocks(M, RS_K)), dim3(RS_T), 0, st, p->key, M, p->perm, p->skey,
                           p->invperm);
    } else {
        const size_t n2 = pow2_at_least((size_t)M, BIT_BLOCK);
        uint64_t* comp = tmp_n<uint64_t>(p, n2);
        hipLaunchKernelGGL(k_composite, dim3(nblocks(n2, 256)), dim3(256), 0, st, p->key, M, n2, comp);
        bitonic_sort(comp, n2, st);
        hipLaunchKernelGGL(k_unpack, dim3(nblocks(M, 256)), dim3(256), 0, st, comp, M, p->perm, p->skey,
                           p->invperm);
    }

    p->cell = alloc_n<int32_t>(p, 3 * (size_t)M);
    p->taps64 = alloc_n<double>(p, 12 * (size_t)M);
    p->taps32 = alloc_n<float>(p, 12 * (size_t)M);
    hipLaunchKernelGGL(k_taps, dim3(nblocks(M, 256)), dim3(256), 0, st, p->perm, cell_c, frac, M, dim,
                       p->delta, p->cell, p->taps64, p->taps32);
    p->line_start = alloc_n<int32_t>(p, (size_t)p->nlines + 1);
    hipLaunchKernelGGL(k_line_start, dim3(nblocks((size_t)p->nlines + 1, 256)), dim3(256), 0, st,
                       p->skey, M, n, p->nlines, p->line_start);

    // spread matrices and line sets: everything up to the sizes on the device, the
    // sizes read back in one copy, then the arrays
    const bool mono = p->bc == IBDL_NEUMANN || p->form != IBDL_FORM_DOUBLE_LAYER;
    const int nl = p->nlines;
    const int32_t* dip_off = csr_count(p, p->dip, true, st);
    // the single layer: Neumann data (S V_b) and the completion (eta S Q)
    const int32_t* mono_off = mono ? csr_count(p, p->mono, false, st) : nullptr;

    int32_t* fl_spread = tmp_n<int32_t>(p, (size_t)nl + 1);
    IBDL_HIP_TRY(hipMemsetAsync(fl_spread, 0, ((size_t)nl + 1) * sizeof(int32_t), st));
    p->spread_line_mask = alloc_n<uint8_t>(p, nl);
    hipLaunchKernelGGL(k_spread_mask, dim3(nblocks(nl, 256)), dim3(256), 0, st, p->dip.line_act, nl,
                       p->spread_line_mask, fl_spread);
    const Compaction c_sl = flag_scan(p, fl_spread, nl, st);

    int32_t* fl_gather = tmp_n<int32_t>(p, (size_t)nl + 1);
    IBDL_HIP_TRY(hipMemsetAsync(fl_gather, 0, ((size_t)nl + 1) * sizeof(int32_t), st));
    p->gather_line_mask = alloc_n<uint8_t>(p, nl);
    IBDL_HIP_TRY(hipMemsetAsync(p->gather_line_mask, 0, nl, st));
    const int per = dim == 3 ? 16 : 4;
    hipLaunchKernelGGL(k_gather_mark, dim3(nblocks((size_t)M * per, 256)), dim3(256), 0, st, p->cell, M,
                       dim, n, p->gather_line_mask);
    hipLaunchKernelGGL(k_mask_to_flag, dim3(nblocks(nl, 256)), dim3(256), 0, st, p->gather_line_mask, nl, fl_gather);
    const Compaction c_gl = flag_scan(p, fl_gather, nl, st);

    Compaction c_sp, c_gp;
    if (dim == 3) {
        int32_t* fl_sp = tmp_n<int32_t>(p, (size_t)n + 1);
        int32_t* fl_gp = tmp_n<int32_t>(p, (size_t)n + 1);
        IBDL_HIP_TRY(hipMemsetAsync(fl_sp, 0, ((size_t)n + 1) * sizeof(int32_t), st));
        IBDL_HIP_TRY(hipMemsetAsync(fl_gp, 0, ((size_t)n + 1) * sizeof(int32_t), st));
        p->spread_plane_mask = alloc_n<uint8_t>(p, n);
        p->gather_plane_mask = alloc_n<uint8_t>(p, n);
        hipLaunchKernelGGL(k_plane_mask, dim3(nblocks(n, 256)), dim3(256), 0, st, p->spread_line_mask, n,
                           p->spread_plane_mask, fl_sp);
        hipLaunchKernelGGL(k_plane_mask, dim3(nblocks(n, 256)), dim3(256), 0, st, p->gather_line_mask, n,
                           p->gather_plane_mask, fl_gp);
        c_sp = flag_scan(p, fl_sp, n, st);
        c_gp = flag_scan(p, fl_gp, n, st);
    }

    CountPtrs cp{};
    cp.p[0] = p->dip.line_act + nl;
    cp.p[1] = dip_off + nl;
    cp.p[2] = mono ? p->mono.line_act + nl : dip_off + nl;
    cp.p[3] = mono ? mono_off + nl : dip_off + nl;
    cp.p[4] = c_sl.idx + nl;
    cp.p[5] = c_gl.idx + nl;
    cp.p[6] = dim == 3 ? c_sp.idx + n : c_sl.idx + nl;
    cp.p[7] = dim == 3 ? c_gp.idx + n : c_gl.idx + nl;
    cp.n = 8;
    int32_t* dcounts = tmp_n<int32_t>(p, 8);
    hipLaunchKernelGGL(k_gather_counts, dim3(1), dim3(64), 0, st, cp, dcounts);
    int32_t hc[8];
    IBDL_HIP_TRY(hipMemcpyAsync(hc, dcounts, sizeof(hc), hipMemcpyDeviceToHost, st));
    IBDL_HIP_TRY(hipStreamSynchronize(st));

    csr_fill(p, p->dip, true, dip_off, hc[0], hc[1], st);
    if (mono) csr_fill(p, p->mono, false, mono_off, hc[2], hc[3], st);
    p->n_spread_lines = hc[4];
    p->spread_lines = compact_list(p, c_sl, hc[4], st);
    p->n_gather_lines = hc[5];
    p->gather_lines = compact_list(p, c_gl, hc[5], st);
    if (dim == 3) {
        p->n_spread_planes = hc[6];
        p->spread_planes = compact_list(p, c_sp, hc[6], st);
        p->n_gather_planes = hc[7];
        p->gather_planes = compact_list(p, c_gp, hc[7], st);
    }

    p->tw64 = alloc_n<double>(p, 2 * (size_t)n);
    p->tw32 = alloc_n<float>(p, 2 * (size_t)n);
    p->s2_64 = alloc_n<double>(p, n);
    p->s2_32 = alloc_n<float>(p, n);
    hipLaunchKernelGGL(k_tables, dim3(nblocks(n, 256)), dim3(256), 0, st, n, p->h, p->length,
                       p->lap == IBDL_LAP_SPECTRAL ? 1 : 0, p->tw64, p->tw32, p->s2_64, p->s2_32);
    if (dim == 2 && p->prec == IBDL_PREC_MIXED) {
        const size_t total = (size_t)tile_pitch_f32(n) * n;
        p->sym32 = alloc_n<float>(p, total);
        hipLaunchKernelGGL(k_symtab, dim3(nblocks(total, 256)), dim3(256), 0, st, n, col_width_f32(n), p->W,
                           total, p->s2_64, p->alpha, 2.0 / ((double)p->nlines * (double)n), p->sym32);
    }
    IBDL_HIP_TRY(hipGetLastError());
    IBDL_HIP_TRY(hipStreamSynchronize(st));
    free_build_tmp(p);
}

void free_build_tmp(ibdl_plan p) {
    for (void* t : p->build_tmp) dev_free(t);
    p->build_tmp.clear();
}

void ensure_workspace(ibdl_plan p, int nrhs) {
    if (p->ws.cap_rhs >= nrhs) return;
    // sized for FP64: mixed plans run their once-per-solve passes in FP64
    const size_t cs = 16;
    const size_t rs = 8;
    // grow: the old buffers are freed in stream order after the work already queued
    // on the plan's stream (a switch of stream waits for the old one first)
    if (p->ws.spec && p->last_stream != alloc_stream()) IBDL_HIP_TRY(hipStreamSynchronize(p->last_stream));
    for (void* old : {p->ws.spec, p->ws.part, p->ws.qf, (void*)p->ws.dmask}) {
        if (!old) continue;
        p->allocs.erase(std::remove(p->allocs.begin(), p->allocs.end(), old), p->allocs.end());
        dev_free(old);
    }
    p->ws.spec = p->ws.part = p->ws.qf = nullptr;
    p->ws.dmask = nullptr;
    p->ws.cap_rhs = 0;
    p->ws.spec = dev_alloc(p, (size_t)nrhs * p->spec_elems * cs);
    p->ws.part = dev_alloc(p, (size_t)nrhs * p->M * p->gpp * rs);
    // packed strengths, four right-hand sides to a segment, in the pass's precision
    p->ws.qf = dev_alloc(p, (size_t)((nrhs + 3) / 4) * 4 * p->M * rs);
    p->ws.dmask = reinterpret_cast<uint8_t*>(dev_alloc(p, (size_t)nrhs * ((size_t)p->nlines + p->n)));
    p->ws.cap_rhs = nrhs;
}

}  // namespace ibdl
