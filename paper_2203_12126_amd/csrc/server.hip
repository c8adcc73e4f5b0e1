// Serving loop: solve requests of different sizes and dimensions are admitted by
// device-memory footprint and slot count, and every request admitted at the same
// scheduling step forms a cohort whose solve (right-hand side, GMRES with FP64
// refinement, grid solution) runs as one resumable task on its own stream.  The
// worker thread advances every cohort whose last wait point has been reached and
// admits new requests as memory and slots free up, so work of requests that
// arrive while others are on the device overlaps with theirs (continuous
// batching).  Each request keeps its own plan and Krylov state on the device; a
// right-hand side's arithmetic does not depend on its cohort, so a result is the
// same alone and in the mix.  Plans are built by a few builder threads, each on
// its own stream, so that the worker keeps advancing running cohorts while new
// geometries are binned and sorted; a cohort starts once all its plans are built,
// its stream ordered after each build by an event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "solve.h"

namespace ibdl {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    ibdl_desc desc{};
    int nrhs = 1;
    const double* data = nullptr;
    const double* g = nullptr;
    double* sol = nullptr;
    double* u = nullptr;
    ibdl_solve_opts o{};
    size_t footprint = 0;
    hipEvent_t inputs_ready = nullptr;  // recorded on the caller's stream at submission
    Clock::time_point t_submit, t_admit, t_done;
    bool done = false;
    int status = IBDL_OK;
    std::string msg;
    std::vector<ibdl_solve_info> info;
    ibdl_plan plan = nullptr;
    int cohort_size = 0;
    // plan construction by a builder thread: 0 queued, 1 built, 2 failed
    std::atomic<int> build_state{0};
    hipEvent_t plan_ready = nullptr;  // recorded on the builder's stream after the build
};

struct Cohort {
    std::vector<std::shared_ptr<Request>> reqs;
    KrylovSet ks;
    Arena arena;
    std::unique_ptr<SolveTask> task;  // set once every plan is built
    int slot = -1;
};

static bool same_opts(const ibdl_solve_opts& a, const ibdl_solve_opts& b) {
    return a.tol == b.tol && a.restart == b.restart && a.maxit == b.maxit && a.true_residual == b.true_residual;
}

}  // namespace ibdl

struct ibdl_server_s {
    int device = 0;
    size_t budget = 0;
    int max_slots = 0;
    std::vector<hipStream_t> streams;  // one per cohort in flight
    std::vector<int> stream_busy;
    std::mutex mu;
    std::condition_variable cv_submit, cv_done;
    std::deque<std::shared_ptr<ibdl::Request>> pending;
    std::map<uint64_t, std::shared_ptr<ibdl::Request>> live;  // until polled complete
    uint64_t next_ticket = 1;
    size_t in_use = 0, peak_in_use = 0;
    int active = 0, peak_active = 0;
    int64_t submitted = 0, completed = 0, cohorts = 0;
    bool stop = false;
    std::thread worker;
    // plan builders
    std::vector<std::thread> builders;
    std::vector<hipStream_t> build_streams;
    std::deque<std::shared_ptr<ibdl::Request>> build_q;
    std::mutex bmu;
    std::condition_variable bcv;
    bool bstop = false;
};

namespace ibdl {

// bytes a request holds while admitted: its plan, workspace and Krylov state,
// plus the argument tables of its cohort
static size_t request_footprint(const ibdl_desc* d, int nrhs, int restart) {
    const size_t f = ibdl_plan_footprint(d, nrhs, restart);
    return f ? f + (size_t)(4u << 20) : 0;
}

static void complete(ibdl_server s, const std::shared_ptr<Request>& r, bool admitted) {
    std::lock_guard<std::mutex> lk(s->mu);
    r->done = true;
    r->t_done = Clock::now();
    if (admitted) {
        s->in_use -= r->footprint;
        s->active -= 1;
    }
    s->completed += 1;
    if (r->inputs_ready) {
        (void)hipEventDestroy(r->inputs_ready);
        r->inputs_ready = nullptr;
    }
    s->cv_done.notify_all();
}

// frees in stream order on the cohort's stream: no wait for other cohorts
static void release_cohort(ibdl_server s, Cohort& c) {
    const hipStream_t st = s->streams[c.slot];
    (void)hipStreamSynchronize(st);
    AllocStream as(st);
    c.task.reset();
    free_krylov(c.ks.w);
    arena_free(c.arena);
    for (auto& r : c.reqs) {
        if (r->plan) release_plan(r->plan, st);
        r->plan = nullptr;
        if (r->plan_ready) (void)hipEventDestroy(r->plan_ready);
        r->plan_ready = nullptr;
    }
}

static void finish_cohort(ibdl_server s, Cohort& c) {
    std::vector<ibdl_solve_info> info(c.ks.R);
    int overall = IBDL_OK;
    c.task->results(info.data(), &overall);
    for (size_t i = 0; i < c.reqs.size(); ++i) {
        Request& r = *c.reqs[i];
        const Inst& in = c.ks.inst[i];
        r.info.assign(info.begin() + in.r0, info.begin() + in.r0 + in.nrhs);
        int worst = IBDL_OK;
        for (const auto& x : r.info) {
            if (x.status == IBDL_ERR_NUMERIC) worst = IBDL_ERR_NUMERIC;
            else if (x.status == IBDL_ERR_NOCONV && worst == IBDL_OK) worst = IBDL_ERR_NOCONV;
        }
        r.status = worst;
        if (worst == IBDL_ERR_NOCONV) r.msg = "GMRES did not reach tol within maxit";
        if (worst == IBDL_ERR_NUMERIC) r.msg = "non-finite residual";
    }
    release_cohort(s, c);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stream_busy[c.slot] = 0;
    }
    for (auto& r : c.reqs) complete(s, r, true);
}

static void fail_cohort(ibdl_server s, Cohort& c, int status, const std::string& msg) {
    for (auto& r : c.reqs) {
        r->status = status;
        r->msg = msg;
        r->info.assign(r->nrhs, ibdl_solve_info{0, -1.0, -1.0, status, 0});
    }
    release_cohort(s, c);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stream_busy[c.slot] = 0;
    }
    for (auto& r : c.reqs) complete(s, r, true);
}

// builder thread: plans of queued requests, on the builder's own stream
static void builder_loop(ibdl_server s, int b) {
    (void)hipSetDevice(s->device);
    const hipStream_t bst = s->build_streams[b];
    for (;;) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(s->bmu);
            s->bcv.wait(lk, [&] { return s->bstop || !s->build_q.empty(); });
            if (s->build_q.empty()) return;
            r = s->build_q.front();
            s->build_q.pop_front();
        }
        ibdl_plan p = nullptr;
        ibdl_status status = IBDL_OK;
        std::string msg;
        if (hipStreamWaitEvent(bst, r->inputs_ready, 0) != hipSuccess) {
            (void)hipGetLastError();
            status = IBDL_ERR_HIP;
        } else {
            status = ibdl_plan_create(&r->desc, bst, &p);
        }
        if (status != IBDL_OK) msg = ibdl_last_error();
        if (status == IBDL_OK) {
            try {
                AllocStream as(bst);
                ensure_workspace(p, r->nrhs);
                IBDL_HIP_TRY(hipEventCreateWithFlags(&r->plan_ready, hipEventDisableTiming));
                IBDL_HIP_TRY(hipEventRecord(r->plan_ready, bst));
            } catch (const Error& e) {
                release_plan(p, bst);
                p = nullptr;
                status = (ibdl_status)e.status;
                msg = e.msg;
            }
        }
        if (status != IBDL_OK) {
            r->status = status;
            r->msg = msg.empty() ? "plan construction failed" : msg;
        }
        r->plan = p;
        r->build_state.store(status == IBDL_OK ? 1 : 2, std::memory_order_release);
    }
}

// a cohort of admitted requests: their plans go to the builders
static std::unique_ptr<Cohort> queue_cohort(ibdl_server s, std::vector<std::shared_ptr<Request>>& adm, int slot) {
    auto c = std::make_unique<Cohort>();
    c->slot = slot;
    c->ks.arena = &c->arena;
    for (auto& r : adm) r->cohort_size = (int)adm.size();
    c->reqs = adm;
    {
        std::lock_guard<std::mutex> lk(s->bmu);
        for (auto& r : adm) s->build_q.push_back(r);
    }
    s->bcv.notify_all();
    return c;
}

// once every plan of the cohort is built: requests whose build failed complete
// with its error; the others are ordered after their builds and their inputs on
// the cohort's stream and start as one solve task.  false: still building.
static bool start_cohort(ibdl_server s, Cohort& c) {
    for (auto& r : c.reqs)
        if (r->build_state.load(std::memory_order_acquire) == 0) return false;
    const hipStream_t st = s->streams[c.slot];
    std::vector<std::shared_ptr<Request>> ok;
    for (auto& r : c.reqs) {
        if (r->build_state.load(std::memory_order_acquire) == 2) {
            r->info.assign(r->nrhs, ibdl_solve_info{0, -1.0, -1.0, (int32_t)r->status, 0});
            complete(s, r, true);
        } else {
            ok.push_back(r);
        }
    }
    c.reqs = ok;
    if (c.reqs.empty()) return true;
    int r0 = 0;
    for (auto& r : c.reqs) {
        IBDL_HIP_TRY(hipStreamWaitEvent(st, r->plan_ready, 0));
        IBDL_HIP_TRY(hipStreamWaitEvent(st, r->inputs_ready, 0));
        r->plan->last_stream = st;  // the plan's work continues on the cohort's stream
        c.ks.inst.push_back(Inst{r->plan, r->nrhs, r0});
        r0 += r->nrhs;
    }
    c.ks.R = r0;
    SolveIO io;
    for (auto& r : c.reqs) {
        io.data.push_back(r->data);
        io.g.push_back(r->g);
        io.x0.push_back(nullptr);
        io.sol.push_back(r->sol);
        io.u.push_back(r->u);
        io.vb.push_back(r->desc.bc == IBDL_NEUMANN ? r->data : nullptr);
    }
    c.task = std::make_unique<SolveTask>(c.ks, std::move(io), c.reqs[0]->o, st);
    c.task->advance();
    return true;
}

static void server_loop(ibdl_server s) {
    (void)hipSetDevice(s->device);
    std::vector<std::unique_ptr<Cohort>> cohorts;
    for (;;) {
        std::vector<std::shared_ptr<Request>> adm;
        int slot = -1;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->stop && s->pending.empty() && cohorts.empty()) break;
            for (size_t i = 0; i < s->stream_busy.size(); ++i)
                if (!s->stream_busy[i]) {
                    slot = (int)i;
                    break;
                }
            // first come, first served: the head of the queue waits for memory
            // and slots; requests behind it do not overtake it
            while (slot >= 0 && !s->pending.empty() && s->active < s->max_slots) {
                auto& r = s->pending.front();
                if (!adm.empty() && !same_opts(adm[0]->o, r->o)) break;
                if (s->in_use + r->footprint > s->budget) break;
                s->in_use += r->footprint;
                s->active += 1;
                r->t_admit = Clock::now();
                adm.push_back(r);
                s->pending.pop_front();
            }
            s->peak_in_use = std::max(s->peak_in_use, s->in_use);
            s->peak_active = std::max(s->peak_active, s->active);
            if (!adm.empty()) {
                s->stream_busy[slot] = 1;
                s->cohorts += 1;
            } else if (cohorts.empty()) {
                s->cv_submit.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
        }
        if (!adm.empty()) cohorts.push_back(queue_cohort(s, adm, slot));
        bool progressed = !adm.empty();
        for (size_t i = 0; i < cohorts.size();) {
            Cohort& c = *cohorts[i];
            bool finished = false;
            try {
                if (!c.task) {
                    if (start_cohort(s, c)) {
                        progressed = true;
                        if (!c.task) {  // every build failed
                            std::lock_guard<std::mutex> lk(s->mu);
                            s->stream_busy[c.slot] = 0;
                            finished = true;
                        }
                    }
                }
                while (c.task && !c.task->done() && c.task->ready()) {
                    c.task->advance();
                    progressed = true;
                }
                if (c.task && c.task->done()) {
                    finish_cohort(s, c);
                    finished = true;
                }
            } catch (const Error& e) {
                fail_cohort(s, c, e.status, e.msg);
                finished = true;
            }
            if (finished) {
                cohorts.erase(cohorts.begin() + i);
                progressed = true;
            } else {
                ++i;
            }
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace ibdl

using namespace ibdl;

namespace {
ibdl_status sfail(int status, const std::string& msg) { return ibdl::set_error(status, msg); }
}  // namespace

extern "C" {

ibdl_status ibdl_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t streams, ibdl_server* out) {
    if (!out) return sfail(IBDL_ERR_ARG, "out is NULL");
    if (max_slots < 1) return sfail(IBDL_ERR_ARG, "max_slots must be >= 1");
    if (streams < 1 || streams > 16) return sfail(IBDL_ERR_ARG, "streams must be in 1..16");
    ibdl_server s = new (std::nothrow) ibdl_server_s();
    if (!s) return sfail(IBDL_ERR_OOM, "host allocation failed");
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return sfail(IBDL_ERR_HIP, "no current device");
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        delete s;
        return sfail(IBDL_ERR_HIP, "hipMemGetInfo failed");
    }
    s->budget = hbm_budget_bytes ? hbm_budget_bytes : free_b / 10 * 9;
    if (s->budget > free_b) {
        delete s;
        return sfail(IBDL_ERR_OOM, "budget exceeds the free device memory");
    }
    s->max_slots = max_slots;
    for (int i = 0; i < streams; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
            delete s;
            return sfail(IBDL_ERR_HIP, "stream creation failed");
        }
        s->streams.push_back(st);
        s->stream_busy.push_back(0);
    }
    constexpr int kBuilders = 3;
    for (int i = 0; i < kBuilders; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
            for (hipStream_t t : s->build_streams) (void)hipStreamDestroy(t);
            delete s;
            return sfail(IBDL_ERR_HIP, "stream creation failed");
        }
        s->build_streams.push_back(st);
    }
    try {
        for (int i = 0; i < kBuilders; ++i) s->builders.emplace_back(builder_loop, s, i);
        s->worker = std::thread(server_loop, s);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->bmu);
            s->bstop = true;
        }
        s->bcv.notify_all();
        for (auto& t : s->builders)
            if (t.joinable()) t.join();
        for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
        for (hipStream_t t : s->build_streams) (void)hipStreamDestroy(t);
        delete s;
        return sfail(IBDL_ERR_HIP, "worker thread could not start");
    }
    *out = s;
    return IBDL_OK;
}

ibdl_status ibdl_server_destroy(ibdl_server s) {
    if (!s) return sfail(IBDL_ERR_ARG, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_submit.notify_all();
    if (s->worker.joinable()) s->worker.join();  // every cohort, built or not, has finished
    {
        std::lock_guard<std::mutex> lk(s->bmu);
        s->bstop = true;
    }
    s->bcv.notify_all();
    for (auto& t : s->builders)
        if (t.joinable()) t.join();
    for (hipStream_t t : s->build_streams) (void)hipStreamSynchronize(t);
    for (hipStream_t t : s->build_streams) (void)hipStreamDestroy(t);
    for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
    delete s;
    return IBDL_OK;
}

ibdl_status ibdl_server_footprint(const ibdl_desc* desc, int32_t nrhs, int32_t restart, size_t* bytes) {
    if (!bytes) return sfail(IBDL_ERR_ARG, "bytes is NULL");
    *bytes = request_footprint(desc, nrhs, restart);
    return *bytes ? IBDL_OK : sfail(IBDL_ERR_ARG, "invalid desc, nrhs or restart");
}

ibdl_status ibdl_server_submit(ibdl_server s, const ibdl_desc* desc, int32_t nrhs, const double* data,
                               const double* g, const ibdl_solve_opts* opts, double* sol, double* u,
                               void* stream, uint64_t* ticket) {
    if (!s) return sfail(IBDL_ERR_ARG, "server is NULL");
    if (!ticket) return sfail(IBDL_ERR_ARG, "ticket is NULL");
    if (!desc || nrhs < 1) return sfail(IBDL_ERR_ARG, "desc must be set and nrhs >= 1");
    if (!data || !sol) return sfail(IBDL_ERR_ARG, "data and sol must be device pointers");
    ibdl_solve_opts o{1e-8, 50, 500, nullptr, 0};
    if (opts) o = *opts;
    if (!(o.tol > 0.0)) return sfail(IBDL_ERR_ARG, "tol must be positive");
    if (o.restart < 1 || o.restart > 200) return sfail(IBDL_ERR_ARG, "restart must be in 1..200");
    if (o.maxit < 1) return sfail(IBDL_ERR_ARG, "maxit must be >= 1");
    if (o.x0) return sfail(IBDL_ERR_ARG, "opts->x0 must be NULL for served solves");
    if (desc->form != IBDL_FORM_DOUBLE_LAYER) return sfail(IBDL_ERR_ARG, "servers take the double-layer formulation");
    const size_t fp = request_footprint(desc, nrhs, o.restart);
    if (!fp) return sfail(IBDL_ERR_ARG, "invalid desc");
    if (fp > s->budget) return sfail(IBDL_ERR_OOM, "request footprint exceeds the server's memory budget");
    auto r = std::make_shared<Request>();
    r->desc = *desc;
    r->nrhs = nrhs;
    r->data = data;
    r->g = g;
    r->sol = sol;
    r->u = u;
    r->o = o;
    r->footprint = fp;
    if (hipEventCreateWithFlags(&r->inputs_ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(r->inputs_ready, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        if (r->inputs_ready) (void)hipEventDestroy(r->inputs_ready);
        return sfail(IBDL_ERR_HIP, "could not record the inputs' event");
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            (void)hipEventDestroy(r->inputs_ready);
            return sfail(IBDL_ERR_STATE, "server is shutting down");
        }
        r->ticket = s->next_ticket++;
        s->pending.push_back(r);
        s->live[r->ticket] = r;
        s->submitted += 1;
    }
    s->cv_submit.notify_all();
    *ticket = r->ticket;
    return IBDL_OK;
}

static ibdl_status take_result(ibdl_server s, std::unique_lock<std::mutex>& lk, uint64_t ticket,
                               ibdl_solve_info* info, ibdl_request_times* times) {
    auto it = s->live.find(ticket);
    auto r = it->second;
    s->live.erase(it);
    lk.unlock();
    if (info)
        for (int i = 0; i < r->nrhs; ++i) info[i] = r->info[i];
    if (times) {
        using ms = std::chrono::duration<double, std::milli>;
        times->queue_ms = ms(r->t_admit - r->t_submit).count();
        times->run_ms = ms(r->t_done - r->t_admit).count();
        times->total_ms = ms(r->t_done - r->t_submit).count();
        times->cohort_size = r->cohort_size;
    }
    if (r->status != IBDL_OK) return sfail(r->status, r->msg);
    return IBDL_OK;
}

ibdl_status ibdl_server_poll(ibdl_server s, uint64_t ticket, ibdl_solve_info* info, ibdl_request_times* times) {
    if (!s) return sfail(IBDL_ERR_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return sfail(IBDL_ERR_ARG, "unknown ticket");
    if (!it->second->done) return IBDL_ERR_STATE;
    return take_result(s, lk, ticket, info, times);
}

ibdl_status ibdl_server_wait(ibdl_server s, uint64_t ticket, ibdl_solve_info* info, ibdl_request_times* times) {
    if (!s) return sfail(IBDL_ERR_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return sfail(IBDL_ERR_ARG, "unknown ticket");
    auto r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    return take_result(s, lk, ticket, info, times);
}

ibdl_status ibdl_server_get_stats(ibdl_server s, ibdl_server_stats* out) {
    if (!s || !out) return sfail(IBDL_ERR_ARG, "server and out must not be NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->cohorts = s->cohorts;
    out->pending = (int32_t)s->pending.size();
    out->active = s->active;
    out->peak_active = s->peak_active;
    out->in_use_bytes = s->in_use;
    out->peak_in_use_bytes = s->peak_in_use;
    out->budget_bytes = s->budget;
    return IBDL_OK;
}

}  // extern "C"
