// C ABI of the IBDL library: argument checks, error reporting, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "plan.h"

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
    if (d->npts < 1) return "npts must be >= 1";
    const long long per = d->dim == 2 ? 32 : 160;
    if ((long long)d->npts * per >= (1LL << 31)) return "too many boundary points";
    if (!d->X || !d->normal || !d->weight) return "X, normal and weight must be device pointers";
    return "";
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
}  // namespace

namespace ibdl {

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

void* ring_put(JobRing& r, const void* src, size_t bytes, hipStream_t st) {
    const size_t need = (bytes + 255) / 256 * 256;
    if (!r.host || need > r.cap) {
        if (r.host) IBDL_HIP_TRY(hipStreamSynchronize(st));
        const size_t cap = std::max<size_t>(need, 4u << 20);
        void* h = nullptr;
        IBDL_HIP_TRY(hipHostMalloc(&h, cap));
        if (r.host) (void)hipHostFree(r.host);
        r.host = reinterpret_cast<char*>(h);
        r.dev = reinterpret_cast<char*>(dev_alloc(*r.owner, cap));
        r.cap = cap;
        r.pos = 0;
    }
    if (r.pos + need > r.cap) {
        // wrap: copies queued earlier must have consumed the host staging area
        IBDL_HIP_TRY(hipStreamSynchronize(st));
        r.pos = 0;
    }
    std::memcpy(r.host + r.pos, src, bytes);
    IBDL_HIP_TRY(hipMemcpyAsync(r.dev + r.pos, r.host + r.pos, bytes, hipMemcpyHostToDevice, st));
    void* d = r.dev + r.pos;
    r.pos += need;
    return d;
}

static void flush_set(ibdl_plan p, int set) {
    const int n = p->set_used[set];
    if (n <= 0) return;
    IBDL_HIP_TRY(hipEventSynchronize(p->ev[set][2 * n - 1]));
    for (int i = 0; i < n; ++i) {
        float ms = 0.f;
        IBDL_HIP_TRY(hipEventElapsedTime(&ms, p->ev[set][2 * i], p->ev[set][2 * i + 1]));
        const char* nm = p->set_names[set][i];
        int slot = -1;
        for (int k = 0; k < p->n_acc; ++k)
            if (std::strcmp(p->acc_names[k], nm) == 0) slot = k;
        if (slot < 0 && p->n_acc < 16) {
            slot = p->n_acc++;
            p->acc_names[slot] = nm;
            p->acc_ms[slot] = 0.0;
            p->acc_n[slot] = 0;
        }
        if (slot >= 0) {
            p->acc_ms[slot] += ms;
            p->acc_n[slot] += 1;
        }
    }
    p->set_used[set] = 0;
}

// Stage names must be string literals.
StageEv stage_events(ibdl_plan p, int idx, const char* name) {
    StageEv e;
    if (!p->timing || idx >= ibdl_plan_s::MAXST) return e;
    if (!p->events_made) {
        for (int s = 0; s < ibdl_plan_s::RING; ++s)
            for (int i = 0; i < 2 * ibdl_plan_s::MAXST; ++i) IBDL_HIP_TRY(hipEventCreate(&p->ev[s][i]));
        p->events_made = 1;
    }
    if (idx == 0) {
        const int set = p->ring_pos;
        flush_set(p, set);
        p->cur_set = set;
        p->ring_pos = (set + 1) % ibdl_plan_s::RING;
    }
    if (p->cur_set < 0) return e;
    p->set_names[p->cur_set][idx] = name;
    p->set_used[p->cur_set] = idx + 1;
    e.a = p->ev[p->cur_set][2 * idx];
    e.b = p->ev[p->cur_set][2 * idx + 1];
    return e;
}

void apply_operator(ibdl_plan p, int nrhs, const double* q, size_t qstride, double* out, size_t ostride,
                    hipStream_t st) {
    // A q = -S* L^-1 S~ q + s q/2, s = +1 Dirichlet, -1 Neumann
    PipeIn in;
    in.q_dip = q;
    in.c_dip = 1.0;
    in.q_stride = qstride;
    PipeOut o;
    o.out = out;
    o.out_stride = ostride;
    o.cA = -1.0;
    o.in = q;
    o.in_stride = qstride;
    o.cB = p->bc == IBDL_DIRICHLET ? 0.5 : -0.5;
    run_pipeline(p, nrhs, in, o, st);
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
    p->ring.owner = &p->allocs;
    try {
        p->dim = desc->dim;
        p->n = desc->n;
        p->bc = desc->bc;
        p->delta = desc->delta;
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
    (void)hipDeviceSynchronize();
    for (void* a : p->allocs) (void)hipFree(a);
    if (p->kr.host_pinned) (void)hipHostFree(p->kr.host_pinned);
    if (p->ring.host) (void)hipHostFree(p->ring.host);
    if (p->events_made)
        for (int s = 0; s < ibdl_plan_s::RING; ++s)
            for (int i = 0; i < 2 * ibdl_plan_s::MAXST; ++i) (void)hipEventDestroy(p->ev[s][i]);
    delete p;
    return IBDL_OK;
}

size_t ibdl_plan_footprint(const ibdl_desc* d, int32_t nrhs, int32_t restart) {
    if (!check_desc(d).empty() || nrhs < 1 || restart < 1) return 0;
    const size_t n = d->n, M = d->npts, dim = d->dim;
    const size_t nlines = dim == 2 ? n : n * n;
    const size_t P = (n / 2 + 1 + 15) / 16 * 16;
    const size_t cs = d->prec == IBDL_PREC_FP64 ? 16 : 8;
    const size_t npp = dim == 2 ? 32 : 160;
    size_t b = 0;
    b += (size_t)nrhs * nlines * P * cs;                 // spectra
    b += (size_t)nrhs * M * (dim == 3 ? 16 : 4) * 8;     // partial sums
    const size_t nnz = M * npp;
    size_t n2 = 2048;
    while (n2 < nnz) n2 <<= 1;
    b += n2 * 8 + nnz * (4 + 8 + 4 + 4 + 4);             // sorted keys, weights, scan buffers
    if (d->bc == IBDL_NEUMANN) b += nnz / 2 * 24;
    b += M * (4 * 6 + 12 * 12 + 8 * 4) + nlines * 24;   // geometry, taps, tables, lists
    b += (size_t)nrhs * ((restart + 1) * M * 8 + 3 * M * 8 + (restart + 2) * (restart + 8) * 8);
    return b;
}

ibdl_status ibdl_apply(ibdl_plan p, int32_t nrhs, const double* q, double* Aq, void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!q || !Aq) return fail(IBDL_ERR_ARG, "q and Aq must be device pointers");
    if (q == Aq) return fail(IBDL_ERR_ARG, "q and Aq must not overlap");
    IBDL_GUARD_BEGIN
    apply_operator(p, nrhs, q, (size_t)p->M, Aq, (size_t)p->M, S(stream));
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_rhs(ibdl_plan p, int32_t nrhs, const double* data, const double* g, double* b,
                     void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!data || !b) return fail(IBDL_ERR_ARG, "data and b must be device pointers");
    IBDL_GUARD_BEGIN
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

ibdl_status ibdl_solve(ibdl_plan p, int32_t nrhs, const double* data, const double* g,
                       const ibdl_solve_opts* opts, double* sol, ibdl_solve_info* info, void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!data || !sol) return fail(IBDL_ERR_ARG, "data and sol must be device pointers");
    ibdl_solve_opts o{1e-8, 50, 500, nullptr, 0};
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(IBDL_ERR_ARG, "tol must be positive");
    if (o.restart < 1 || o.restart > 200) return fail(IBDL_ERR_ARG, "restart must be in 1..200");
    if (o.maxit < 1) return fail(IBDL_ERR_ARG, "maxit must be >= 1");
    IBDL_GUARD_BEGIN
    int overall = IBDL_OK;
    gmres_solve(p, nrhs, data, g, o, sol, info, S(stream), &overall);
    if (overall == IBDL_ERR_NOCONV) return fail(IBDL_ERR_NOCONV, "GMRES did not reach tol within maxit");
    if (overall == IBDL_ERR_NUMERIC) return fail(IBDL_ERR_NUMERIC, "non-finite residual");
    g_last_error.clear();
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_eval_grid(ibdl_plan p, int32_t nrhs, const double* sol, const double* vb,
                           const double* g, double* u, void* stream) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    if (nrhs < 1) return fail(IBDL_ERR_ARG, "nrhs must be >= 1");
    if (!sol || !u) return fail(IBDL_ERR_ARG, "sol and u must be device pointers");
    if (p->bc == IBDL_NEUMANN && !vb) return fail(IBDL_ERR_ARG, "Neumann plans need V_b");
    IBDL_GUARD_BEGIN
    PipeIn in;
    in.q_dip = sol;
    in.c_dip = -1.0;
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
    return IBDL_OK;
}

ibdl_status ibdl_plan_set_timing(ibdl_plan p, int32_t enable) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    IBDL_GUARD_BEGIN
    for (int s = 0; s < ibdl_plan_s::RING; ++s) p->set_used[s] = 0;
    p->n_acc = 0;
    p->cur_set = -1;
    p->ring_pos = 0;
    p->timing = enable ? 1 : 0;
    return IBDL_OK;
    IBDL_GUARD_END
}

ibdl_status ibdl_plan_stage_times(ibdl_plan p, double* ms_host, const char** names, int64_t* calls,
                                  int32_t cap, int32_t* count) {
    if (!p) return fail(IBDL_ERR_ARG, "plan is NULL");
    IBDL_GUARD_BEGIN
    for (int s = 0; s < ibdl_plan_s::RING; ++s) flush_set(p, s);
    for (int i = 0; i < p->n_acc && i < cap; ++i) {
        if (ms_host) ms_host[i] = p->acc_n[i] ? p->acc_ms[i] / (double)p->acc_n[i] : 0.0;
        if (names) names[i] = p->acc_names[i];
        if (calls) calls[i] = p->acc_n[i];
    }
    if (count) *count = p->n_acc;
    return IBDL_OK;
    IBDL_GUARD_END
}

}  // extern "C"
