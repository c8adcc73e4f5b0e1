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

// scans in, or the flags in > 0 when positive is set
__global__ __launch_bounds__(SCAN_T) void k_scan_tile(const int32_t* in, int32_t* out, size_t n,
                                                      int32_t* sums, int positive) {
    __shared__ int32_t s[SCAN_T];
    const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_PER;
    int32_t v[SCAN_PER];
    int32_t tot = 0;
    for (int i = 0; i < SCAN_PER; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        if (positive) v[i] = v[i] > 0;
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

// out = exclusive scan of in (n entries), or of the flags in > 0 with positive set;
// the total is out[n-1] plus the last entry (or flag)
static void scan_excl(ibdl_plan p, const int32_t* in, int32_t* out, size_t n, hipStream_t st, bool positive = false) {
    const size_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nt <= 1) {
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(SCAN_T), 0, st, in, out, n, (int32_t*)nullptr,
                           positive ? 1 : 0);
        return;
    }
    int32_t* sums = tmp_n<int32_t>(p, nt);
    int32_t* soff = tmp_n<int32_t>(p, nt);
    hipLaunchKernelGGL(k_scan_tile, dim3((int)nt), dim3(SCAN_T), 0, st, in, out, n, sums, positive ? 1 : 0);
    scan_excl(p, sums, soff, nt, st);
    hipLaunchKernelGGL(k_scan_add, dim3(nblocks(n, 256)), dim3(256), 0, st, out, n, soff);
}

static int32_t read_i32(const int32_t* d, hipStream_t st) {
    int32_t v = 0;
    IBDL_HIP_TRY(hipMemcpyAsync(&v, d, sizeof(v), hipMemcpyDeviceToHost, st));
    IBDL_HIP_TRY(hipStreamSynchronize(st));
    return v;
}

__global__ void k_sum2(const int32_t* a, const int32_t* b, int32_t* out) { *out = *a + *b; }

// a count from an exclusive scan: its last entry plus the last flag, read with one wait
static int32_t read_count(ibdl_plan p, const int32_t* scan_last, const int32_t* flag_last, hipStream_t st) {
    int32_t* d = tmp_n<int32_t>(p, 1);
    hipLaunchKernelGGL(k_sum2, dim3(1), dim3(1), 0, st, scan_last, flag_last, d);
    return read_i32(d, st);
}

// ------------------------------------------------------------------ sorted geometry
// Rank sort for small point counts: the sorted position of point k is the number of
// composites (key << 32 | index) below its own -- all distinct, so the ranks are a
// permutation and equal keys keep the caller order.  A block ranks RS_K points,
// RS_SPLIT threads per point each counting over a quarter of every tile of RS_T.
constexpr int RS_K = 64, RS_SPLIT = 4, RS_T = RS_K * RS_SPLIT;
constexpr int RANK_SORT_MAX = 16384;  // above this the bitonic sort is faster

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
// Stencil offsets r in -2..3 (dipole) or -1..2 (monopole) per axis; the dipole
// keeps the nodes where at most one axis offset lies outside -1..2 (elsewhere
// every term of div(S q n) vanishes).
// Offsets of the dipole stencil's nodes from a point's cell, in order: the boxes of
// 6^dim around it whose weight is structurally nonzero (at most one axis outside
// -1..2, where the centred difference reaches one node further): 32 in 2-D, 160 in 3-D
struct DipStencil {
    int8_t o[160][3];
};
constexpr DipStencil dip_stencil(int dim) {
    DipStencil t{};
    int cnt = 0;
    const int tot = dim == 2 ? 36 : 216;
    for (int b = 0; b < tot; ++b) {
        const int o0 = b % 6 - 2, o1 = (b / 6) % 6 - 2, o2 = dim == 3 ? b / 36 - 2 : 0;
        const int outside = (o0 < -1 || o0 > 2) + (o1 < -1 || o1 > 2) + (o2 < -1 || o2 > 2);
        if (outside <= 1) {
            t.o[cnt][0] = (int8_t)o0;
            t.o[cnt][1] = (int8_t)o1;
            t.o[cnt][2] = (int8_t)o2;
            ++cnt;
        }
    }
    return t;
}
__constant__ DipStencil kDip2 = dip_stencil(2);
__constant__ DipStencil kDip3 = dip_stencil(3);

// node id of stencil entry j of the point at sorted position s
__device__ __forceinline__ uint32_t stencil_node(const int32_t* __restrict__ cell_s, int s, int j, int dim, int n,
                                                 int dipole) {
    int r[3] = {0, 0, 0};
    if (dipole) {
        const int8_t* o = dim == 2 ? kDip2.o[j] : kDip3.o[j];
        r[0] = o[0];
        r[1] = o[1];
        r[2] = o[2];
    } else {
        r[0] = j % 4 - 1;
        r[1] = (j / 4) % 4 - 1;
        r[2] = dim == 3 ? j / 16 - 1 : 0;
    }
    uint32_t node = 0, stride = 1;
    for (int d = 0; d < dim; ++d) {
        // cell in [0, n), offset in -2..3, n >= 8: one periodic wrap at most
        int c = cell_s[3 * s + d] + r[d];
        c += c < 0 ? n : 0;
        c -= c >= n ? n : 0;
        node += (uint32_t)c * stride;
        stride *= (uint32_t)n;
    }
    return node;
}

// entries per grid node: every (point, stencil node) pair counts once
__global__ void k_node_count(const int32_t* __restrict__ cell_s, int M, int dim, int n, int dipole, int npp,
                             int32_t* cnt) {
    // M * npp < 2^31 (checked by the caller): 32-bit index arithmetic
    const int id = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (id >= M * npp) return;
    const int s = id / npp;
    atomicAdd(&cnt[stencil_node(cell_s, s, id - s * npp, dim, n, dipole)], 1);
}

__global__ void k_flag_of(const int32_t* cnt, int32_t* flag) { *flag = *cnt > 0; }

// active nodes in ascending id and their entry counts; idx = exclusive scan of the flags
__global__ void k_compact_nodes(const int32_t* __restrict__ cnt, const int32_t* __restrict__ idx, size_t ncell,
                                uint32_t* act_node, int32_t* act_cnt) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell || cnt[c] == 0) return;
    act_node[idx[c]] = (uint32_t)c;
    act_cnt[idx[c]] = cnt[c];
}

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

// The cells c = p - r, r in [rlo, rhi], of one axis in ascending (periodic) order:
// start at the first unwrapped offset u0 + t whose wrapped value is the smallest
struct AxisRun {
    int u0, cnt, t0;
};
__device__ __forceinline__ AxisRun axis_run(int p, int rlo, int rhi, int n) {
    AxisRun a;
    a.u0 = p - rhi;
    a.cnt = rhi - rlo + 1;
    const int ulast = p - rlo;
    a.t0 = a.u0 < 0 ? -a.u0 : (ulast >= n ? n - a.u0 : 0);
    return a;
}
__device__ __forceinline__ int axis_cell(const AxisRun& a, int i, int n) {
    int t = a.t0 + i;
    t -= t >= a.cnt ? a.cnt : 0;
    int c = a.u0 + t;
    c += c < 0 ? n : 0;
    c -= c >= n ? n : 0;
    return c;
}

// first sorted position in [s0, s1) of x-line points whose cell x is >= cx (skey % n
// ascends within a line)
__device__ __forceinline__ int line_lower(const uint32_t* __restrict__ skey, int s0, int s1, int n, int cx) {
    while (s0 < s1) {
        const int mid = (s0 + s1) >> 1;
        if ((int)(skey[mid] % (uint32_t)n) < cx) s0 = mid + 1; else s1 = mid;
    }
    return s0;
}

// One active node per thread: its entries are the points of the cells c = node - r
// over the stencil offsets r.  A row of cells along x at fixed (y, z) is one or two
// ranges of sorted positions, found in the x-line's points.  Writes the caller index
// and the node's active index of each entry, in the order found; a count that
// differs from the node's raises bad[3] and writes nothing past the node's range.
__global__ void k_fill(const uint32_t* __restrict__ act_node, const int32_t* __restrict__ act_ptr, int nact,
                       int dim, int n, int dipole, const int32_t* __restrict__ line_start,
                       const uint32_t* __restrict__ skey, const uint32_t* __restrict__ perm, uint32_t* ent_k,
                       int32_t* ent_a, int32_t* bad) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nact) return;
    const uint32_t node = act_node[a];
    const int pc[3] = {(int)(node % (uint32_t)n), (int)((node / (uint32_t)n) % (uint32_t)n),
                       dim == 3 ? (int)(node / ((uint32_t)n * (uint32_t)n)) : 0};
    const int e0 = act_ptr[a], e1 = act_ptr[a + 1];
    int e = e0;
    // offsets per axis: dipole -2..3 with at most one axis outside -1..2, monopole -1..2
    const int lo = dipole ? -2 : -1, hi = dipole ? 3 : 2;
    const AxisRun rz = dim == 3 ? axis_run(pc[2], lo, hi, n) : AxisRun{0, 1, 0};
    const AxisRun ry = axis_run(pc[1], lo, hi, n);
    for (int iz = 0; iz < rz.cnt; ++iz) {
        const int cz = dim == 3 ? axis_cell(rz, iz, n) : 0;
        const int oz = dim == 3 ? ((pc[2] - cz + 2 + 2 * n) % n) - 2 : 0;
        for (int iy = 0; iy < ry.cnt; ++iy) {
            const int cy = axis_cell(ry, iy, n);
            const int oy = ((pc[1] - cy + 2 + 2 * n) % n) - 2;
            const int outside = (oy < -1 || oy > 2) + (oz < -1 || oz > 2);
            if (outside > 1) continue;
            const int line = cz * n + cy;
            const int l0 = line_start[line], l1 = line_start[line + 1];
            if (l0 == l1) continue;
            const int xlo = outside ? -1 : lo, xhi = outside ? 2 : hi;
            // cells pc[0] - xhi .. pc[0] - xlo along x: one range, or two across the seam
            const int u0 = pc[0] - xhi, u1 = pc[0] - xlo;
            int seg[2][2];
            int nseg = 1;
            if (u0 < 0) {
                seg[0][0] = 0; seg[0][1] = u1; seg[1][0] = u0 + n; seg[1][1] = n - 1; nseg = 2;
            } else if (u1 >= n) {
                seg[0][0] = 0; seg[0][1] = u1 - n; seg[1][0] = u0; seg[1][1] = n - 1; nseg = 2;
            } else {
                seg[0][0] = u0; seg[0][1] = u1;
            }
            for (int g = 0; g < nseg; ++g) {
                const int s0 = line_lower(skey, l0, l1, n, seg[g][0]);
                const int s1 = line_lower(skey, s0, l1, n, seg[g][1] + 1);
                if (e + (s1 - s0) > e1) {
                    bad[3] = 1;
                    return;
                }
                for (int s = s0; s < s1; ++s, ++e) {
                    ent_k[e] = perm[s];
                    ent_a[e] = a;
                }
            }
        }
    }
    if (e != e1) bad[3] = 1;
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

// entry weights, one entry per thread (K: the entries' caller indices, ent_a: their
// nodes' active indices)
__global__ void k_entry_weights(size_t nnz, const int32_t* __restrict__ ent_a,
                                const uint32_t* __restrict__ act_node, int dim, int n,
                                const int32_t* __restrict__ cell_s, const uint32_t* __restrict__ invperm,
                                const double* __restrict__ taps64, const double* __restrict__ nrm3,
                                const double* __restrict__ w1, double h, int dipole, const uint32_t* __restrict__ K,
                                double* W64, float* W32) {
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
    W64[e] = wv;
    W32[e] = (float)wv;
}

__global__ void k_set_i32(int32_t* p, int32_t v) { *p = v; }

// first active node index with node / n >= line
__global__ void k_line_act(const uint32_t* __restrict__ act_node, int nact, int n, int nlines,
                           int32_t* la) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > nlines) return;
    int lo = 0, hi = nact;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)(act_node[mid] / (uint32_t)n) < l) lo = mid + 1; else hi = mid;
    }
    la[l] = lo;
}

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
static int compact(ibdl_plan p, const int32_t* flag, int n, int32_t** list, hipStream_t st) {
    int32_t* idx = tmp_n<int32_t>(p, (size_t)n + 1);
    scan_excl(p, flag, idx, (size_t)n, st);
    const int cnt = read_count(p, idx + n - 1, flag + n - 1, st);
    *list = alloc_n<int32_t>(p, (size_t)std::max(cnt, 1));
    hipLaunchKernelGGL(k_compact_list, dim3(nblocks(n, 256)), dim3(256), 0, st, flag, idx, n, *list);
    return cnt;
}

// Dense per-node counts and their flag scan, shared by the spread matrices of one plan
struct CsrScratch {
    size_t ncell = 0;
    int32_t* cnt = nullptr;  // [ncell]
    int32_t* idx = nullptr;  // [ncell]
    int32_t* bad = nullptr;
};

static void build_csr(ibdl_plan p, Csr& c, bool dipole, const CsrScratch& cs, hipStream_t st) {
    const int dim = p->dim, n = p->n, M = p->M;
    const int npp = dipole ? (dim == 2 ? 32 : 160) : (dim == 2 ? 16 : 64);
    const size_t nnz = (size_t)M * npp;
    if (nnz * sizeof(double) >= (size_t)INT32_MAX) throw Error{IBDL_ERR_ARG, "too many spread entries"};
    const size_t ncell = cs.ncell;
    // rows: nodes with at least one entry, ascending; their counts and offsets
    IBDL_HIP_TRY(hipMemsetAsync(cs.cnt, 0, ncell * sizeof(int32_t), st));
    hipLaunchKernelGGL(k_node_count, dim3(nblocks(nnz, 256)), dim3(256), 0, st, p->cell, M, dim, n,
                       dipole ? 1 : 0, npp, cs.cnt);
    scan_excl(p, cs.cnt, cs.idx, ncell, st, true);
    // flag of the last node: its count, positive or zero (read_count adds it as is)
    int32_t* last_flag = tmp_n<int32_t>(p, 1);
    hipLaunchKernelGGL(k_flag_of, dim3(1), dim3(1), 0, st, cs.cnt + ncell - 1, last_flag);
    c.nact = read_count(p, cs.idx + ncell - 1, last_flag, st);
    c.act_node = alloc_n<uint32_t>(p, (size_t)std::max(c.nact, 1));
    c.act_ptr = alloc_n<int32_t>(p, (size_t)c.nact + 1);
    int32_t* act_cnt = tmp_n<int32_t>(p, (size_t)std::max(c.nact, 1));
    hipLaunchKernelGGL(k_compact_nodes, dim3(nblocks(ncell, 256)), dim3(256), 0, st, cs.cnt, cs.idx, ncell,
                       c.act_node, act_cnt);
    scan_excl(p, act_cnt, c.act_ptr, (size_t)c.nact, st);
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, st, c.act_ptr + c.nact, (int32_t)nnz);
    // entries, collected per node from the x-lines around it (no sort of the entries),
    // then weighed one per thread
    c.nnz = (int64_t)nnz;
    c.k = alloc_n<uint32_t>(p, nnz);
    c.w64 = alloc_n<double>(p, nnz);
    c.w32 = alloc_n<float>(p, nnz);
    uint32_t* ent_k = tmp_n<uint32_t>(p, nnz);
    int32_t* ent_a = tmp_n<int32_t>(p, nnz);
    hipLaunchKernelGGL(k_fill, dim3(nblocks(c.nact, 256)), dim3(256), 0, st, c.act_node, c.act_ptr, c.nact, dim, n,
                       dipole ? 1 : 0, p->line_start, p->skey, p->perm, ent_k, ent_a, cs.bad);
    hipLaunchKernelGGL(k_entry_order, dim3(nblocks(nnz, 256)), dim3(256), 0, st, nnz, ent_k, ent_a, c.act_ptr, c.k);
    hipLaunchKernelGGL(k_entry_weights, dim3(nblocks(nnz, 256)), dim3(256), 0, st, nnz, ent_a, c.act_node, dim, n,
                       p->cell, p->invperm, p->taps64, p->nrm, p->wgt, p->h, dipole ? 1 : 0, c.k, c.w64, c.w32);
    c.line_act = alloc_n<int32_t>(p, (size_t)p->nlines + 1);
    hipLaunchKernelGGL(k_line_act, dim3(nblocks((size_t)p->nlines + 1, 256)), dim3(256), 0, st,
                       c.act_node, c.nact, n, p->nlines, c.line_act);
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

    // per-node counts, shared by the spread matrices
    CsrScratch cs;
    cs.ncell = (size_t)p->nlines * n;
    cs.cnt = tmp_n<int32_t>(p, cs.ncell);
    cs.idx = tmp_n<int32_t>(p, cs.ncell);
    cs.bad = bad;
    build_csr(p, p->dip, true, cs, st);
    // the single layer: Neumann data (S V_b) and the completion (eta S Q)
    if (p->bc == IBDL_NEUMANN || p->form != IBDL_FORM_DOUBLE_LAYER) build_csr(p, p->mono, false, cs, st);

    // line and plane sets
    int32_t* flag = tmp_n<int32_t>(p, (size_t)std::max(p->nlines, n));
    p->spread_line_mask = alloc_n<uint8_t>(p, p->nlines);
    hipLaunchKernelGGL(k_spread_mask, dim3(nblocks(p->nlines, 256)), dim3(256), 0, st, p->dip.line_act,
                       p->nlines, p->spread_line_mask, flag);
    p->n_spread_lines = compact(p, flag, p->nlines, &p->spread_lines, st);

    p->gather_line_mask = alloc_n<uint8_t>(p, p->nlines);
    IBDL_HIP_TRY(hipMemsetAsync(p->gather_line_mask, 0, p->nlines, st));
    const int per = dim == 3 ? 16 : 4;
    hipLaunchKernelGGL(k_gather_mark, dim3(nblocks((size_t)M * per, 256)), dim3(256), 0, st, p->cell, M,
                       dim, n, p->gather_line_mask);
    hipLaunchKernelGGL(k_mask_to_flag, dim3(nblocks(p->nlines, 256)), dim3(256), 0, st,
                       p->gather_line_mask, p->nlines, flag);
    p->n_gather_lines = compact(p, flag, p->nlines, &p->gather_lines, st);

    if (dim == 3) {
        p->spread_plane_mask = alloc_n<uint8_t>(p, n);
        p->gather_plane_mask = alloc_n<uint8_t>(p, n);
        hipLaunchKernelGGL(k_plane_mask, dim3(nblocks(n, 256)), dim3(256), 0, st, p->spread_line_mask, n,
                           p->spread_plane_mask, flag);
        p->n_spread_planes = compact(p, flag, n, &p->spread_planes, st);
        hipLaunchKernelGGL(k_plane_mask, dim3(nblocks(n, 256)), dim3(256), 0, st, p->gather_line_mask, n,
                           p->gather_plane_mask, flag);
        p->n_gather_planes = compact(p, flag, n, &p->gather_planes, st);
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
    IBDL_HIP_TRY(hipMemcpyAsync(hb, bad, sizeof(hb), hipMemcpyDeviceToHost, st));
    IBDL_HIP_TRY(hipStreamSynchronize(st));
    if (hb[3]) throw Error{IBDL_ERR_STATE, "internal: spread matrix entry count mismatch"};
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
    for (void* old : {p->ws.spec, p->ws.part, p->ws.qf}) {
        if (!old) continue;
        p->allocs.erase(std::remove(p->allocs.begin(), p->allocs.end(), old), p->allocs.end());
        dev_free(old);
    }
    p->ws.spec = p->ws.part = p->ws.qf = nullptr;
    p->ws.cap_rhs = 0;
    p->ws.spec = dev_alloc(p, (size_t)nrhs * p->spec_elems * cs);
    p->ws.part = dev_alloc(p, (size_t)nrhs * p->M * p->gpp * rs);
    if (p->prec == IBDL_PREC_MIXED) p->ws.qf = dev_alloc(p, (size_t)((nrhs + 3) / 4) * 4 * p->M * sizeof(float));
    p->ws.cap_rhs = nrhs;
}

}  // namespace ibdl
