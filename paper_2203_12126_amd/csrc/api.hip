// C ABI of the IBDL library: argument checks, error reporting, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>

#include "solve.h"

namespace {
thread_local std::string g_last_error;

ibdl_status fail(int status, const std::string& msg) {
    g_last_error = msg;
    return (ibdl_status)status;
}

bool size_ok(int n) {
    if (n < 8) return false;
    int t = n;
    while (t % 2 == 0) t /= 2;
    while (t % 3 == 0) t /= 3;
    return t == 1;
}

const int kSizes[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048};

bool supported_n(int dim, int n) {
    bool listed = false;
    for (int s : kSizes) listed |= (s == n);
    if (!listed || !size_ok(n)) return false;
    return dim == 2 ? n <= 2048 : n <= 512;
}

std::string check_desc(const ibdl_desc* d) {
    if (!d) return "desc is NULL";
    if (d->dim != 2 && d->dim != 3) return "dim must be 2 or 3";
    if (!supported_n(d->dim, d->n))
        return "n must be one of 8,12,16,24,32,48,64,96,128,192,256,384,512,768,1024,1536,2048 "
               "(<= 512 in 3-D)";
    for (int i = 0; i < d->dim; ++i)
        if (!std::isfinite(d->lo[i])) return "lo must be finite";
    if (!(d->length > 0.0) || !std::isfinite(d->length)) return "length must be positive and finite";
    if (!(d->alpha >= 0.0) || !std::isfinite(d->alpha)) return "alpha must be >= 0 and finite";
    if (d->bc != IBDL_DIRICHLET && d->bc != IBDL_NEUMANN) return "bc must be IBDL_DIRICHLET or IBDL_NEUMANN";
    if (d->delta != IBDL_DELTA_PESKIN4 && d->delta != IBDL_DELTA_COSINE4) return "unknown delta kernel";
    if (d->prec != IBDL_PREC_FP64 && d->prec != IBDL_PREC_MIXED) return "unknown precision";
    if (d->lap != IBDL_LAP_FD && d->lap != IBDL_LAP_SPECTRAL) return "lap must be IBDL_LAP_FD or IBDL_LAP_SPECTRAL";
    if (d->form != IBDL_FORM_DOUBLE_LAYER && d->form != IBDL_FORM_COMPLETED && d->form != IBDL_FORM_SINGLE_LAYER)
        return "unknown formulation";
    if (d->form == IBDL_FORM_SINGLE_LAYER) {
        if (d->bc != IBDL_DIRICHLET) return "the single-layer formulation takes Dirichlet data";
        if (d->prec != IBDL_PREC_FP64) return "the single-layer formulation runs in FP64";
    }
    if (d->form == IBDL_FORM_COMPLETED) {
        if (d->alpha != 0.0) return "the completed formulation is for the Poisson equation (alpha = 0)";
        if (d->bc != IBDL_DIRICHLET) return "the completed formulation takes Dirichlet data";
        if (!(d->eta > 0.0) || !std::isfinite(d->eta)) return "eta must be positive and finite";
    }
    if (d->npts < 1) return "npts must be >= 1";
    // spread entries per point (dipole stencil); the spread kernels address the
    // entries' FP64 weights with 32-bit byte offsets
    const long long per = d->dim == 2 ? 32 : 160;
    if ((long long)d->npts * per * 8 >= (1LL << 31)) return "too many boundary points";
    if (!d->X || !d->normal || !d->weight) return "X, normal and weight must be device pointers";
    return "";
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
}  // namespace

namespace ibdl {

ibdl_status set_error(int status, const std::string& msg) { return fail(status, msg); }

std::unique_ptr<PreparedPass> prepare_pass(const std::vector<PassJob>& jobs, bool fp64) {
    for (const PassJob& j : jobs) ensure_workspace(j.p, j.nrhs);
    if (fp64 || jobs[0].p->prec == IBDL_PREC_FP64) return prepare_f64(jobs);
    return prepare_f32(jobs);
}

void run_pipeline(ibdl_plan p, int nrhs, const PipeIn& in, const PipeOut& out, hipStream_t st,
                  bool fp64) {
    std::vector<PassJob> jobs{PassJob{p, nrhs, in, out}};
    prepare_pass(jobs, fp64)->run(0, st);
}

void arena_flush(Arena& a, hipStream_t st) {
    if (a.cur < (int)a.blocks.size() && a.pos > a.pend) {
        Arena::Block& blk = a.blocks[a.cur];
        IBDL_HIP_TRY(hipMemcpyAsync(blk.dev + a.pend, blk.host + a.pend, a.pos - a.pend, hipMemcpyHostToDevice, st));
    }
    a.pend = a.pos;
}

void* arena_put(Arena& a, const void* src, size_t bytes, hipStream_t st) {
    void* d = arena_stage(a, src, bytes, st);
    arena_flush(a, st);
    return d;
}

void* arena_stage(Arena& a, const void* src, size_t bytes, hipStream_t st) {
    const size_t need = (bytes + 255) / 256 * 256;
    if (a.cur < (int)a.blocks.size() && a.pos + need > a.blocks[a.cur].cap) arena_flush(a, st);
    while (a.cur < (int)a.blocks.size() && a.pos + need > a.blocks[a.cur].cap) {
        ++a.cur;
        a.pos = 0;
        a.pend = 0;
    }
    if (a.cur == (int)a.blocks.size()) {
        Arena::Block blk;
        blk.cap = std::max<size_t>(need, 4u << 20);
        blk.host = reinterpret_cast<char*>(pinned_get(blk.cap));
        std::vector<void*> own;
        try {
            blk.dev = reinterpret_cast<char*>(dev_alloc(own, blk.cap));
        } catch (...) {
            pinned_put(blk.host);
            throw;
        }
        a.blocks.push_back(blk);
        a.pos = 0;
        a.pend = 0;
    }
    Arena::Block& blk = a.blocks[a.cur];
    std::memcpy(blk.host + a.pos, src, bytes);
    void* d = blk.dev + a.pos;
    a.pos += need;
    return d;
}

void arena_reset(Arena& a) {
    a.cur = 0;
    a.pos = 0;
    a.pend = 0;
}

void arena_free(Arena& a) {
    for (auto& b : a.blocks) {
        dev_free(b.dev);
        pinned_put(b.host);
    }
    a.blocks.clear();
    a.cur = 0;
    a.pos = 0;
    a.pend = 0;
}

static void flush_set(Timing& t, int set) {
    const int n = t.set_used[set];
    if (n <= 0) return;
    IBDL_HIP_TRY(hipEventSynchronize(t.ev[set][2 * n - 1]));
    for (int i = 0; i < n; ++i) {
        float ms = 0.f;
        IBDL_HIP_TRY(hipEventElapsedTime(&ms, t.ev[set][2 * i], t.ev[set][2 * i + 1]));
        const char* nm = t.set_names[set][i];
        int slot = -1;
        for (int k = 0; k < t.n_acc; ++k)
            if (std::strcmp(t.acc_names[k], nm) == 0) slot = k;
        if (slot < 0 && t.n_acc < 16) {
            slot = t.n_acc++;
            t.acc_names[slot] = nm;
            t.acc_ms[slot] = 0.0;
            t.acc_n[slot] = 0;
        }
        if (slot >= 0) {
            t.acc_ms[slot] += ms;
            t.acc_n[slot] += 1;
        }
    }
    t.set_used[set] = 0;
}

// Stage names must be string literals.
StageEv stage_events(ibdl_plan p, int idx, const char* name) {
    StageEv e;
    Timing& t = *p->tm;
    if (!t.enabled || idx >= Timing::MAXST) return e;
    if (!t.events_made) {
        for (int s = 0; s < Timing::RING; ++s)
            for (int i = 0; i < 2 * Timing::MAXST; ++i) IBDL_HIP_TRY(hipEventCreate(&t.ev[s][i]));
        t.events_made = 1;
    }
    if (idx == 0) {
        const int set = t.ring_pos;
        flush_set(t, set);
        t.cur_set = set;
        t.ring_pos = (set + 1) % Timing::RING;
    }
    if (t.cur_set < 0) return e;
    t.set_names[t.cur_set][idx] = name;
    t.set_used[t.cur_set] = idx + 1;
    e.a = t.ev[t.cur_set][2 * idx];
    e.b = t.ev[t.cur_set][2 * idx + 1];
    return e;
}

void timing_reset(Timing& t, int enable) {
    for (int s = 0; s < Timing::RING; ++s) t.set_used[s] = 0;
    t.n_acc = 0;
    t.cur_set = -1;
    t.ring_pos = 0;
    t.enabled = enable ? 1 : 0;
}

void timing_free(Timing& t) {
    if (t.events_made)
        for (int s = 0; s < Timing::RING; ++s)
            for (int i = 0; i < 2 * Timing::MAXST; ++i) (void)hipEventDestroy(t.ev[s][i]);
    t.events_made = 0;
}

int timing_read(Timing& t, double* ms, const char** names, int64_t* calls, int cap) {
    for (int s = 0; s < Timing::RING; ++s) flush_set(t, s);
    for (int i = 0; i < t.n_acc && i < cap; ++i) {
        if (ms) ms[i] = t.acc_n[i] ? t.acc_ms[i] / (double)t.acc_n[i] : 0.0;
        if (names) names[i] = t.acc_names[i];
        if (calls) calls[i] = t.acc_n[i];
    }
    return t.n_acc;
}

void apply_operator(ibdl_plan p, int nrhs, const double* q, size_t qstride, double* out, size_t ostride,
                    hipStream_t st, bool pack_q) {
    // A q = -S* L^-1 S~ q + s q/2, s = +1 Dirichlet, -1 Neumann
    PipeIn in;
    in.q_dip = q;
    in.c_dip = 1.0;
    in.q_stride = qstride;
    // passes of several right-hand sides over a large spread read the strengths
    // packed four right-hand sides to a segment in the pass's precision (the values
    // the spread rounds them to: results do not change)
    in.pack_q = pack_q;
    PipeOut o;
    o.out = out;
    o.out_stride = ostride;
    o.cA = -1.0;
    o.in = q;
    o.in_stride = qstride;
    o.cB = p->bc == IBDL_DIRICHLET ? 0.5 : -0.5;
    run_pipeline(p, nrhs, in, o, st);
}

// ------------------------------------------------------------------ allocation-free apply
// The device scratch of ibdl_apply_noalloc: the half spectra and gather partial
// sums of its pass.  Each device that loads the library holds its own copy until
// the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

// the current device's scratch address, looked up once per device
static char* scratch_base() {
    int dev = 0;
    IBDL_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error{IBDL_ERR_HIP, "device index beyond the scratch table"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        IBDL_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Error{IBDL_ERR_HIP, "hipGetSymbolAddress gave no scratch address"};
        g_scratch_dev[dev] = ptr;
    }
    return reinterpret_cast<char*>(g_scratch_dev[dev]);
}

// bytes of scratch the pass of ibdl_apply_noalloc needs: spectra and partials in
// the precision of the plan's operator pass, each part 256-byte aligned
static size_t noalloc_bytes(ibdl_plan p, int nrhs, size_t* spec_bytes) {
    const bool f64 = p->prec == IBDL_PREC_FP64;
    const size_t cs = f64 ? 16 : 8, rs = f64 ? 8 : 4;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t sb = up((size_t)nrhs * p->spec_elems * cs);
    if (spec_bytes) *spec_bytes = sb;
    return sb + up((size_t)nrhs * p->M * p->gpp * rs);
}

// ------------------------------------------------------------------ tile autotuner
namespace {
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, float>> g_tune;
std::atomic<int> g_tune_on{1};
}  // namespace

int tune_lookup(const TuneKey& k) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(k);
    return it == g_tune.end() ? -1 : it->second.first;
}
void tune_store(const TuneKey& k, int variant, float ms) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[k] = {variant, ms};
}
bool tune_enabled() { return g_tune_on.load() == 1; }
int tune_forced() {
    const int m = g_tune_on.load();
    return m >= 2 ? m - 2 : -1;
}

bool& capturing() {
    thread_local bool c = false;
    return c;
}

namespace {
std::atomic<int> g_graphs_on{0};
std::atomic<int64_t> g_graphs_recorded{0}, g_graph_replays{0};
}  // namespace
bool graphs_enabled() { return g_graphs_on.load() != 0; }
void note_graphs(int64_t recorded, int64_t replays) {
    g_graphs_recorded += recorded;
    g_graph_replays += replays;
}

void release_plan(ibdl_plan p, hipStream_t st) {
    AllocStream as(st);
    free_build_tmp(p);
    for (void* a : p->allocs) dev_free(a);
    p->allocs.clear();
    free_krylov(p->ks.w);
    arena_free(p->arena);
    timing_free(p->own_timing);
    delete p;
}

}  // namespace ibdl

using namespace ibdl;

#define IBDL_GUARD_BEGIN try {
#define IBDL_GUARD_END                                                        \
    }                                                                         \
    catch (const ibdl::Error& e) { return fail(e.status, e.msg); }            \
    catch (const std::bad_alloc&) { return fail(IBDL_ERR_OOM, "host allocation failed"); } \
    catch (...) { return fail(IBDL_ERR_HIP, "unexpected failure"); }

extern "C" {

const char* ibdl_last_error(void) { return g_last_error.c_str(); }

ibdl_status ibdl_plan_create(const ibdl_desc* desc, void* stream, ibdl_plan* out) {
    if (!out) return fail(IBDL_ERR_ARG, "out is NULL");
    const std::string why = check_desc(desc);
    if (!why.empty()) return fail(IBDL_ERR_ARG, why);
    ibdl_plan p = new (std::nothrow) ibdl_plan_s();
    if (!p) return fail(IBDL_ERR_OOM, "host allocation failed");
    AllocStream as(S(stream));
    p->last_stream = S(stream);
    p->ks.arena = &p->arena;
    try {
        p->dim = desc->dim;
        p->n = desc->n;
        p->bc = desc->bc;
        p->delta = desc->delta;
        p->lap = desc->lap;
        p->form = desc->form;
        p->eta = desc->form == IBDL_FORM_COMPLETED ? desc->eta : 0.0;
        p->prec = desc->prec;
        p->M = desc->npts;
        for (int i = 0; i < 3; ++i) p->lo[i] = i < desc->dim ? desc->lo[i] : 0.0;
        p->length = desc->length;
        p->h = desc->length / desc->n;
        p->alpha = desc->alpha;
        p->W = desc->n / 2 + 1;
        p->P = std::max(tile_pitch_f64(desc->n), tile_pitch_f32(desc->n));
        p->nlines = desc->dim == 2 ? desc->n : desc->n * desc->n;
        p->spec_elems = (size_t)p->nlines * p->P;
        p->gpp = desc->dim == 3 ? 16 : 4;
        build_plan(p, desc, S(stream));
    } catch (const ibdl::Error& e) {
        ibdl_plan_destroy(p);
        return fail(e.status, e.msg);
    } catch (...) {
        ibdl_plan_destroy(p);
        return fail(IBDL_ERR_HIP, "plan construction failed");
    }
    *out = p;
    g_last_error.clear();
    return IBDL_OK;
}

ibdl_status ibdl_plan_destroy(ibdl_plan p) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    // the plan may have been used on several streams: wait for the device, then free
    (void)hipDeviceSynchronize();
    release_plan(p, nullptr);
    return IBDL_OK;
}

size_t ibdl_plan_footprint(const ibdl_desc* d, int32_t nrhs, int32_t restart) {
    if (!check_desc(d).empty() || nrhs < 1 || restart < 1) return 0;
    const size_t n = d->n, M = d->npts, dim = d->dim, R = nrhs, m = restart;
    const size_t nlines = dim == 2 ? n : n * n;
    const size_t P = (size_t)std::max(tile_pitch_f64(d->n), tile_pitch_f32(d->n));
    const size_t gpp = dim == 3 ? 16 : 4;
    auto pow2 = [](size_t v) {
        size_t t = 2048;
        while (t < v) t <<= 1;
        return t;
    };
    size_t b = 0;
    // workspace, FP64-sized: half spectra and gather partial sums
    b += R * nlines * P * 16 + R * M * gpp * 8 + R * (nlines + n);
    // packed strengths in groups of four right-hand sides (FP64-sized)
    b += (R + 3) / 4 * 4 * M * 8;
    // sorted geometry: key, perm, skey, invperm, cell, coordinates, normals, weights, taps (FP64 + FP32)
    b += M * (16 + 12 + 24 + 24 + 8 + 96 + 48);
    // spread structures (entry: point as caller index and sorted position, FP64 and
    // FP32 weight; active node id and offset)
    const size_t nd = M * (dim == 2 ? 32 : 160);
    const size_t nm = (d->bc == IBDL_NEUMANN || d->form != IBDL_FORM_DOUBLE_LAYER) ? M * (dim == 2 ? 16 : 64) : 0;
    b += (nd + nm) * 28 + 2 * (nlines + 2) * 4;
    // line and plane masks, lists, line starts, FFT and symbol tables
    b += nlines * 18 + n * 64;
    if (dim == 2 && d->prec == IBDL_PREC_MIXED) b += (size_t)tile_pitch_f32(d->n) * n * 4;
    // construction temporaries, alive together at most: the points' sort keys, line
    // counts and their scans (two spread matrices), line and plane flags and scans,
    // the entries as found (point and node), scan partials
    b += M * 36 + pow2(M) * 8 + (nd + nm) * 8 + (nlines + 1) * 4 * 10 + (n + 1) * 4 * 4 +
         (nlines / 256 + 64) * 8 * 8;
    // Krylov state: basis, five pools, two banks of block partial sums, Hessenberg and rotations
    const size_t nblk = (M + 255) / 256;
    b += R * ((m + 1) * M * 8 + 5 * M * 8 + 2 * nblk * (m + 2) * 8 + (m * (m + 1) + 4 * m + 3 * (m + 2)) * 8 + 64);
    // allocation granularity: small buffers, and the device's 2 MiB pages (one more
    // page for buffers that straddle them)
    // completed formulation: Q2, the per-call Q1 and sums, grid-sum partials
    if (d->form == IBDL_FORM_COMPLETED) b += (M + 1) * 8 + R * (M + 2) * 8 + R * 256 * 8 + 3 * 4096;
    // single-layer formulation: the nine MINRES vectors, block partials and scalars
    if (d->form == IBDL_FORM_SINGLE_LAYER) b += R * (9 * M * 8 + ((M + 255) / 256) * 8 + 14 * 8 + 16) + 13 * 4096;
    b += 96 * 4096;
    const size_t page = (size_t)2 << 20;
    return (b + page - 1) / page * page + page;
}

ibdl_status ibdl_apply(ibdl_plan p, int32_t nrhs, const double* q, double* Aq, void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!q || !Aq) return fail(IBDL_ERR_ARG, "q and Aq must be device pointers");
    if (q == Aq) return fail(IBDL_ERR_ARG, "q and Aq must not overlap");
    IBDL_GUARD_BEGIN
    AllocStream as(S(stream));
    p->last_stream = S(stream);
    if (p->form == IBDL_FORM_COMPLETED) {
        completed_apply(p, nrhs, q, Aq, S(stream));
        return IBDL_OK;
    }
    if (p->form == IBDL_FORM_SINGLE_LAYER) {
        ibsl_apply(p, nrhs, q, Aq, S(stream));
        return IBDL_OK;
    }
    apply_operator(p, nrhs, q, (size_t)p->M, Aq, (size_t)p->M, S(stream), true);
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_apply_noalloc(ibdl_plan p, int32_t nrhs, const double* q, double* Aq, void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!q || !Aq) return fail(IBDL_ERR_ARG, "q and Aq must be device pointers");
    if (q == Aq) return fail(IBDL_ERR_ARG, "q and Aq must not overlap");
    if (p->form != IBDL_FORM_DOUBLE_LAYER)
        return fail(IBDL_ERR_ARG, "ibdl_apply_noalloc takes plans of the double-layer formulation");
    size_t spec_b = 0;
    const size_t need = noalloc_bytes(p, nrhs, &spec_b);
    if (need > kScratchBytes)
        return fail(IBDL_ERR_ARG, "ibdl_apply_noalloc: " + std::to_string(nrhs) + " right-hand sides of this plan need " +
                                      std::to_string(need) + " bytes of scratch, more than its " +
                                      std::to_string(kScratchBytes) + " (use fewer right-hand sides per call)");
    IBDL_GUARD_BEGIN
    char* base = scratch_base();
    // the pass reads its workspace from the plan: point it at the scratch for this
    // call (the kernels take the addresses at launch) and restore it afterwards;
    // untuned row shapes take the fixed rule instead of timing every shape
    const Workspace saved = p->ws;
    const bool was_capturing = capturing();
    p->ws.spec = base;
    p->ws.part = base + spec_b;
    p->ws.qf = nullptr;
    p->ws.dmask = nullptr;
    p->ws.cap_rhs = nrhs;
    capturing() = true;
    try {
        // no packed strengths: their buffer is not part of the scratch
        apply_operator(p, nrhs, q, (size_t)p->M, Aq, (size_t)p->M, S(stream), false);
    } catch (...) {
        p->ws = saved;
        capturing() = was_capturing;
        throw;
    }
    p->ws = saved;
    capturing() = was_capturing;
    p->last_stream = S(stream);
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_rhs(ibdl_plan p, int32_t nrhs, const double* data, const double* g, double* b,
                     void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!data || !b) return fail(IBDL_ERR_ARG, "data and b must be device pointers");
    IBDL_GUARD_BEGIN
    AllocStream as(S(stream));
    p->last_stream = S(stream);
    if (p->form == IBDL_FORM_COMPLETED) {
        completed_rhs(p, nrhs, data, g, b, S(stream));
        return IBDL_OK;
    }
    PipeIn in;
    PipeOut out;
    out.out = b;
    if (p->bc == IBDL_DIRICHLET) {
        in.grid = g;
        in.c_grid = 1.0;
        out.cA = -1.0;
        out.in = data;
        out.cB = 1.0;
        if (!g) {
            IBDL_HIP_TRY(hipMemcpyAsync(b, data, (size_t)nrhs * p->M * sizeof(double),
                                        hipMemcpyDeviceToDevice, S(stream)));
            return IBDL_OK;
        }
    } else {
        in.q_mono = data;
        in.c_mono = 1.0;
        in.grid = g;
        in.c_grid = -1.0;
        out.cA = 1.0;
    }
    run_pipeline(p, nrhs, in, out, S(stream), true);
    return IBDL_OK;
    IBDL_GUARD_END
}

static ibdl_status plan_solve(ibdl_plan p, int32_t nrhs, const double* data, const double* g,
                              const ibdl_solve_opts* opts, double* sol, double* u, ibdl_solve_info* info,
                              void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!data || !sol) return fail(IBDL_ERR_ARG, "data and sol must be device pointers");
    ibdl_solve_opts o{1e-8, 50, 500, nullptr, 0};
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(IBDL_ERR_ARG, "tol must be positive");
    if (o.restart < 1 || o.restart > 200) return fail(IBDL_ERR_ARG, "restart must be in 1..200");
    if (o.maxit < 1) return fail(IBDL_ERR_ARG, "maxit must be >= 1");
    if (p->form != IBDL_FORM_DOUBLE_LAYER && o.x0)
        return fail(IBDL_ERR_ARG, "opts->x0 must be NULL for completed and single-layer plans");
    IBDL_GUARD_BEGIN
    AllocStream as(S(stream));
    p->last_stream = S(stream);
    int overall = IBDL_OK;
    if (p->form != IBDL_FORM_DOUBLE_LAYER) {
        overall = p->form == IBDL_FORM_COMPLETED ? completed_solve(p, nrhs, data, g, o, sol, u, info, S(stream))
                                                 : ibsl_solve(p, nrhs, data, g, o, sol, u, info, S(stream));
        if (overall == IBDL_ERR_NOCONV) return fail(IBDL_ERR_NOCONV, "GMRES did not reach tol within maxit");
        if (overall == IBDL_ERR_NUMERIC) return fail(IBDL_ERR_NUMERIC, "non-finite residual");
        g_last_error.clear();
        return IBDL_OK;
    }
    p->ks.inst.assign(1, Inst{p, nrhs, 0});
    p->ks.R = nrhs;
    solve_set(p->ks, {data}, {g}, {o.x0}, o, {sol}, info, S(stream), &overall, {u});
    if (overall == IBDL_ERR_NOCONV) return fail(IBDL_ERR_NOCONV, "GMRES did not reach tol within maxit");
    if (overall == IBDL_ERR_NUMERIC) return fail(IBDL_ERR_NUMERIC, "non-finite residual");
    g_last_error.clear();
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_solve(ibdl_plan p, int32_t nrhs, const double* data, const double* g,
                       const ibdl_solve_opts* opts, double* sol, ibdl_solve_info* info, void* stream) {
    return plan_solve(p, nrhs, data, g, opts, sol, nullptr, info, stream);
}

ibdl_status ibdl_solve_grid(ibdl_plan p, int32_t nrhs, const double* data, const double* g,
                            const ibdl_solve_opts* opts, double* sol, double* u, ibdl_solve_info* info,
                            void* stream) {
    if (!u) return fail(IBDL_ERR_ARG, "u must be a device pointer");
    return plan_solve(p, nrhs, data, g, opts, sol, u, info, stream);
}

ibdl_status ibdl_eval_grid(ibdl_plan p, int32_t nrhs, const double* sol, const double* vb,
                           const double* g, double* u, void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!sol || !u) return fail(IBDL_ERR_ARG, "sol and u must be device pointers");
    if (p->bc == IBDL_NEUMANN && !vb) return fail(IBDL_ERR_ARG, "Neumann plans need V_b");
    IBDL_GUARD_BEGIN
    AllocStream as(S(stream));
    p->last_stream = S(stream);
    if (p->form == IBDL_FORM_COMPLETED) {
        completed_eval_grid(p, nrhs, sol, g, u, S(stream));
        return IBDL_OK;
    }
    if (p->form == IBDL_FORM_SINGLE_LAYER) {
        ibsl_eval_grid(p, nrhs, sol, g, u, S(stream));
        return IBDL_OK;
    }
    PipeIn in;
    in.q_dip = sol;
    in.c_dip = -1.0;
    in.pack_q = true;
    if (p->bc == IBDL_NEUMANN) {
        in.q_mono = vb;
        in.c_mono = -1.0;
    }
    in.grid = g;
    in.c_grid = 1.0;
    PipeOut out;
    out.u = u;
    run_pipeline(p, nrhs, in, out, S(stream), true);
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_indicator(ibdl_plan p, double* chi, uint8_t* flags, void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (!chi || !flags) return fail(IBDL_ERR_ARG, "chi and flags must be device pointers");
    IBDL_GUARD_BEGIN
    AllocStream as(S(stream));
    p->last_stream = S(stream);
    nearfix_indicator(p, chi, flags, S(stream));
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_fixup(ibdl_plan p, int32_t nrhs, const double* u, const double* ub, const uint8_t* flags,
                       double m1, double m2, double* u_out, void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!u || !ub || !flags || !u_out) return fail(IBDL_ERR_ARG, "u, ub, flags and u_out must be device pointers");
    if (u == u_out) return fail(IBDL_ERR_ARG, "u and u_out must not overlap");
    if (!(m1 > 0.0) || !std::isfinite(m1) || !(m2 > m1) || !std::isfinite(m2))
        return fail(IBDL_ERR_ARG, "widths must satisfy 0 < m1 < m2");
    if (m2 > 0.25 * p->n) return fail(IBDL_ERR_ARG, "m2 must stay below a quarter of the grid");
    IBDL_GUARD_BEGIN
    AllocStream as(S(stream));
    p->last_stream = S(stream);
    nearfix_fixup(p, nrhs, u, ub, flags, m1, m2, u_out, S(stream));
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_plan_binning(ibdl_plan p, uint32_t* key_host, uint32_t* perm_host) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    IBDL_GUARD_BEGIN
    if (key_host) IBDL_HIP_TRY(hipMemcpy(key_host, p->key, p->M * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (perm_host)
        IBDL_HIP_TRY(hipMemcpy(perm_host, p->perm, p->M * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_plan_get_stats(ibdl_plan p, ibdl_plan_stats* o) {
    if (!p || !o) return fail(IBDL_ERR_ARG, "plan and out must not be NULL");
    o->nlines = p->nlines;
    o->pitch = p->P;
    o->n_spread_lines = p->n_spread_lines;
    o->n_gather_lines = p->n_gather_lines;
    o->n_spread_planes = p->n_spread_planes;
    o->n_gather_planes = p->n_gather_planes;
    o->dip_active_nodes = p->dip.nact;
    o->dip_nnz = p->dip.nnz;
    o->mono_nnz = p->mono.nnz;
    const bool f32 = p->prec == IBDL_PREC_MIXED;
    o->col_tile = f32 ? col_width_f32(p->n) : col_width_f64(p->n);
    o->z_rows = p->dim == 3 ? (f32 ? z_rows_f32(p->n) : z_rows_f64(p->n)) : 1;
    return IBDL_OK;
}

ibdl_status ibdl_plan_set_timing(ibdl_plan p, int32_t enable) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    IBDL_GUARD_BEGIN
    timing_reset(*p->tm, enable);
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_plan_stage_times(ibdl_plan p, double* ms_host, const char** names, int64_t* calls,
                                  int32_t cap, int32_t* count) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    IBDL_GUARD_BEGIN
    const int n = timing_read(*p->tm, ms_host, names, calls, cap);
    if (count) *count = n;
    return IBDL_OK;
    IBDL_GUARD_END
}

// ------------------------------------------------------------------ batches
static bool ptr_array_ok(const void* const* a, int n) {
    if (!a) return false;
    for (int i = 0; i < n; ++i)
        if (!a[i]) return false;
    return true;
}

ibdl_status ibdl_batch_create(const ibdl_desc* descs, int32_t count, const int32_t* nrhs, void* stream,
                              ibdl_batch* out) {
    if (!out) return fail(IBDL_ERR_ARG, "out is NULL");
    if (!descs || !nrhs || count < 1) return fail(IBDL_ERR_ARG, "descs and nrhs must hold count >= 1 entries");
    long long R = 0;
    for (int i = 0; i < count; ++i) {
        const std::string why = check_desc(&descs[i]);
        if (!why.empty()) return fail(IBDL_ERR_ARG, "instance " + std::to_string(i) + ": " + why);
        if (descs[i].form != IBDL_FORM_DOUBLE_LAYER)
            return fail(IBDL_ERR_ARG, "instance " + std::to_string(i) + ": batches take the double-layer formulation");
        if (nrhs[i] < 1) return fail(IBDL_ERR_ARG, "instance " + std::to_string(i) + ": nrhs must be >= 1");
        R += nrhs[i];
    }
    if (R >= (1LL << 24)) return fail(IBDL_ERR_ARG, "too many right-hand sides in one batch");
    ibdl_batch b = new (std::nothrow) ibdl_batch_s();
    if (!b) return fail(IBDL_ERR_OOM, "host allocation failed");
    b->ks.arena = &b->arena;
    b->last_stream = S(stream);
    AllocStream as(S(stream));
    int r0 = 0;
    for (int i = 0; i < count; ++i) {
        ibdl_plan p = nullptr;
        const ibdl_status st = ibdl_plan_create(&descs[i], stream, &p);
        if (st != IBDL_OK) {
            const std::string msg = "instance " + std::to_string(i) + ": " + g_last_error;
            ibdl_batch_destroy(b);
            return fail(st, msg);
        }
        p->tm = &b->timing;
        b->plans.push_back(p);
        b->ks.inst.push_back(Inst{p, nrhs[i], r0});
        r0 += nrhs[i];
    }
    b->ks.R = r0;
    try {
        for (const Inst& in : b->ks.inst) ensure_workspace(in.p, in.nrhs);
    } catch (const ibdl::Error& e) {
        ibdl_batch_destroy(b);
        return fail(e.status, e.msg);
    }
    *out = b;
    g_last_error.clear();
    return IBDL_OK;
}

ibdl_status ibdl_batch_destroy(ibdl_batch b) {
    if (!b) return fail(IBDL_ERR_ARG, "batch is NULL");
    (void)hipDeviceSynchronize();
    AllocStream as(nullptr);
    free_krylov(b->ks.w);
    for (ibdl_plan p : b->plans) release_plan(p, nullptr);
    arena_free(b->arena);
    timing_free(b->timing);
    delete b;
    return IBDL_OK;
}

ibdl_status ibdl_batch_size(ibdl_batch b, int32_t* count, int32_t* total_rhs) {
    if (!b) return fail(IBDL_ERR_ARG, "batch is NULL");
    if (count) *count = (int32_t)b->plans.size();
    if (total_rhs) *total_rhs = b->ks.R;
    return IBDL_OK;
}

ibdl_status ibdl_batch_get_stats(ibdl_batch b, int32_t i, ibdl_plan_stats* out_host) {
    if (!b) return fail(IBDL_ERR_ARG, "batch is NULL");
    if (i < 0 || i >= (int32_t)b->plans.size()) return fail(IBDL_ERR_ARG, "instance index out of range");
    return ibdl_plan_get_stats(b->plans[i], out_host);
}

ibdl_status ibdl_batch_apply(ibdl_batch b, const double* const* q, double* const* Aq, void* stream) {
    if (!b) return fail(IBDL_ERR_ARG, "batch is NULL");
    const int n = (int)b->plans.size();
    if (!ptr_array_ok((const void* const*)q, n) || !ptr_array_ok((const void* const*)Aq, n))
        return fail(IBDL_ERR_ARG, "q and Aq must hold a device pointer per instance");
    for (int i = 0; i < n; ++i)
        if ((const void*)q[i] == (const void*)Aq[i]) return fail(IBDL_ERR_ARG, "q and Aq must not overlap");
    IBDL_GUARD_BEGIN
    IBDL_HIP_TRY(hipStreamSynchronize(S(stream)));
    AllocStream as(S(stream));
    b->last_stream = S(stream);
    arena_reset(b->arena);
    auto make = [&](size_t i) {
        const Inst& in = b->ks.inst[i];
        PipeIn pi;
        pi.q_dip = q[i];
        pi.c_dip = 1.0;
        PipeOut po;
        po.out = Aq[i];
        po.cA = -1.0;
        po.in = q[i];
        po.cB = in.p->bc == IBDL_DIRICHLET ? 0.5 : -0.5;
        return PassJob{in.p, in.nrhs, pi, po};
    };
    std::vector<size_t> all(n);
    for (int i = 0; i < n; ++i) all[i] = i;
    prepare_grouped(b->ks, all, make, false, S(stream)).run(0, S(stream));
    return IBDL_OK;
    IBDL_GUARD_END
}

static ibdl_status batch_solve(ibdl_batch b, const double* const* data, const double* const* g,
                               const ibdl_solve_opts* opts, double* const* sol, double* const* u,
                               ibdl_solve_info* info, void* stream) {
    if (!b) return fail(IBDL_ERR_ARG, "batch is NULL");
    const int n = (int)b->plans.size();
    if (!ptr_array_ok((const void* const*)data, n) || !ptr_array_ok((const void* const*)sol, n))
        return fail(IBDL_ERR_ARG, "data and sol must hold a device pointer per instance");
    ibdl_solve_opts o{1e-8, 50, 500, nullptr, 0};
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(IBDL_ERR_ARG, "tol must be positive");
    if (o.restart < 1 || o.restart > 200) return fail(IBDL_ERR_ARG, "restart must be in 1..200");
    if (o.maxit < 1) return fail(IBDL_ERR_ARG, "maxit must be >= 1");
    if (o.x0) return fail(IBDL_ERR_ARG, "opts->x0 must be NULL for a batch (solves start from 0)");
    IBDL_GUARD_BEGIN
    IBDL_HIP_TRY(hipStreamSynchronize(S(stream)));
    AllocStream as(S(stream));
    b->last_stream = S(stream);
    SolveIO io;
    io.data.assign(data, data + n);
    io.g.assign(n, nullptr);
    if (g) io.g.assign(g, g + n);
    io.sol.assign(sol, sol + n);
    if (u) {
        io.u.assign(u, u + n);
        io.vb = io.data;  // Neumann grid solutions take V_b = the boundary data
    }
    SolveTask t(b->ks, std::move(io), o, S(stream));
    t.run_to_end();
    int overall = IBDL_OK;
    t.results(info, &overall);
    if (overall == IBDL_ERR_NOCONV) return fail(IBDL_ERR_NOCONV, "GMRES did not reach tol within maxit");
    if (overall == IBDL_ERR_NUMERIC) return fail(IBDL_ERR_NUMERIC, "non-finite residual");
    g_last_error.clear();
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_batch_solve(ibdl_batch b, const double* const* data, const double* const* g,
                             const ibdl_solve_opts* opts, double* const* sol, ibdl_solve_info* info,
                             void* stream) {
    return batch_solve(b, data, g, opts, sol, nullptr, info, stream);
}

ibdl_status ibdl_batch_solve_grid(ibdl_batch b, const double* const* data, const double* const* g,
                                  const ibdl_solve_opts* opts, double* const* sol, double* const* u,
                                  ibdl_solve_info* info, void* stream) {
    if (!b) return fail(IBDL_ERR_ARG, "batch is NULL");
    if (!ptr_array_ok((const void* const*)u, (int)b->plans.size()))
        return fail(IBDL_ERR_ARG, "u must hold a device pointer per instance");
    return batch_solve(b, data, g, opts, sol, u, info, stream);
}

ibdl_status ibdl_batch_eval_grid(ibdl_batch b, const double* const* sol, const double* const* vb,
                                 const double* const* g, double* const* u, void* stream) {
    if (!b) return fail(IBDL_ERR_ARG, "batch is NULL");
    const int n = (int)b->plans.size();
    if (!ptr_array_ok((const void* const*)sol, n) || !ptr_array_ok((const void* const*)u, n))
        return fail(IBDL_ERR_ARG, "sol and u must hold a device pointer per instance");
    for (int i = 0; i < n; ++i)
        if (b->plans[i]->bc == IBDL_NEUMANN && (!vb || !vb[i]))
            return fail(IBDL_ERR_ARG, "instance " + std::to_string(i) + ": Neumann instances need V_b");
    IBDL_GUARD_BEGIN
    IBDL_HIP_TRY(hipStreamSynchronize(S(stream)));
    AllocStream as(S(stream));
    b->last_stream = S(stream);
    arena_reset(b->arena);
    auto make = [&](size_t i) {
        const Inst& in = b->ks.inst[i];
        PipeIn pi;
        pi.q_dip = sol[i];
        pi.c_dip = -1.0;
        if (in.p->bc == IBDL_NEUMANN) {
            pi.q_mono = vb[i];
            pi.c_mono = -1.0;
        }
        pi.grid = g ? g[i] : nullptr;
        pi.c_grid = 1.0;
        PipeOut po;
        po.u = u[i];
        return PassJob{in.p, in.nrhs, pi, po};
    };
    std::vector<size_t> all(n);
    for (int i = 0; i < n; ++i) all[i] = i;
    prepare_grouped(b->ks, all, make, true, S(stream)).run(0, S(stream));
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_batch_set_timing(ibdl_batch b, int32_t enable) {
    if (!b) return fail(IBDL_ERR_ARG, "batch is NULL");
    timing_reset(b->timing, enable);
    return IBDL_OK;
}

ibdl_status ibdl_batch_stage_times(ibdl_batch b, double* ms_host, const char** names, int64_t* calls,
                                   int32_t cap, int32_t* count) {
    if (!b) return fail(IBDL_ERR_ARG, "batch is NULL");
    IBDL_GUARD_BEGIN
    const int n = timing_read(b->timing, ms_host, names, calls, cap);
    if (count) *count = n;
    return IBDL_OK;
    IBDL_GUARD_END
}

// ------------------------------------------------------------------ tuning
ibdl_status ibdl_set_autotune(int32_t enable) {
    if (enable < 0 || enable > 5) return set_error(IBDL_ERR_ARG, "ibdl_set_autotune: mode must be 0..5");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_on.store(enable);
    return IBDL_OK;
}

ibdl_status ibdl_set_graphs(int32_t enable) {
    g_graphs_on.store(enable ? 1 : 0);
    return IBDL_OK;
}

ibdl_status ibdl_graph_stats(int64_t* out_host) {
    if (!out_host) return set_error(IBDL_ERR_ARG, "ibdl_graph_stats: null output");
    out_host[0] = g_graphs_recorded.load();
    out_host[1] = g_graph_replays.load();
    return IBDL_OK;
}

int32_t ibdl_autotune_report(char* buf, size_t cap) {
    std::string out;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto& kv : g_tune) {
            const TuneKey& k = kv.first;
            // row-block variants: right-hand sides per block, lines per right-hand side
            static const char* const kVariant[] = {"rhs_per_block=1", "rhs_per_block=2", "rhs_per_block=4",
                                                   "rhs_per_block=1 lines_per_block=1"};
            static const char* const kOut[] = {"points", "grid", "grid+points"};
            const int v = kv.second.first;
            char line[256];
            std::snprintf(line, sizeof(line),
                          "%s dim=%d n=%d stage=%s in=%s out=%s min_rhs_bucket=%d total_rhs_bucket=%d jobs=%s -> %s "
                          "(%.4f ms)\n",
                          k.rbytes == 8 ? "fp64" : "fp32", k.dim, k.n, k.stage == 0 ? "row_fwd" : "row_inv",
                          k.grid_in ? "grid" : "points", kOut[k.dense >= 0 && k.dense <= 2 ? k.dense : 0], k.minr,
                          k.totr, k.multi ? "many" : "one", v >= 0 && v <= 3 ? kVariant[v] : "?",
                          kv.second.second);
            out += line;
        }
    }
    if (buf && cap) {
        const size_t n = std::min(cap - 1, out.size());
        std::memcpy(buf, out.data(), n);
        buf[n] = 0;
    }
    return (int32_t)out.size();
}

}  // extern "C"
