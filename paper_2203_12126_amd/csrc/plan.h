// Internal plan structure of the IBDL library (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/ibdl.h"
#include "common.h"

namespace ibdl {

// Sparse spread operator over the active grid nodes, rows sorted by node id and
// entries within a row by caller point index (a fixed summation order).
struct Csr {
    int64_t nnz = 0;
    int32_t nact = 0;
    uint32_t* act_node = nullptr;   // [nact] flat node id (x fastest)
    int32_t* act_ptr = nullptr;     // [nact+1] first entry of each active node
    uint32_t* k = nullptr;          // [nnz] caller point index
    uint32_t* s = nullptr;          // [nnz] sorted position of the same point
    double* w64 = nullptr;          // [nnz] weight
    float* w32 = nullptr;           // [nnz] weight rounded to FP32
    int32_t* line_act = nullptr;    // [nlines+1] first active node of each x-line
};

struct Workspace {
    int cap_rhs = 0;
    void* spec = nullptr;       // [cap][nlines*P] complex
    void* part = nullptr;       // [cap][M][4^(dim-1)] gather partial sums
    void* qf = nullptr;         // [ceil(cap/4)][M][4] strengths in the plan's precision (FP32 for mixed plans)
    // passes with grid forcing: per right-hand side, 1 for the x-lines whose spectrum
    // the forward row pass wrote ([cap][nlines]), then (3-D) for the z-planes the
    // y pass wrote ([cap][n]); the column passes read only those
    uint8_t* dmask = nullptr;
};

// Staging of per-job argument tables: pinned host blocks with device twins.
// Space is handed out in order and only reclaimed by arena_reset, which the
// caller issues when nothing queued on the stream still reads the tables.
struct Arena {
    struct Block {
        char* host = nullptr;
        char* dev = nullptr;
        size_t cap = 0;
    };
    std::vector<Block> blocks;
    int cur = 0;
    size_t pos = 0;
    size_t pend = 0;  // blocks[cur] bytes [pend, pos) are staged on the host, not yet copied
};
// arena_put: stage and copy at once; arena_stage: host side only, the device
// copies of everything staged since the last flush go out as one copy per block
// in arena_flush, which must precede any launch that reads them
void* arena_put(Arena& a, const void* src, size_t bytes, hipStream_t st);
void* arena_stage(Arena& a, const void* src, size_t bytes, hipStream_t st);
void arena_flush(Arena& a, hipStream_t st);
void arena_reset(Arena& a);
void arena_free(Arena& a);

// One instance of a Krylov set: a plan and its right-hand sides r0 .. r0+nrhs-1.
struct Inst {
    ibdl_plan p = nullptr;
    int nrhs = 0;
    int r0 = 0;
};

struct GroupedPass;

// Device state of restarted GMRES for R right-hand sides of possibly different
// lengths: rhs r has M_r unknowns, basis block voff[r] in V (cap_m+1 vectors),
// vectors xoff[r] in the pools b, x, r, rr, d.
struct KWork {
    int cap_m = 0, R = 0, nblk = 0;
    std::vector<std::pair<ibdl_plan, int>> layout;  // (plan, nrhs) per instance
    double* V = nullptr;
    double* H = nullptr;        // [R][m][m+1] (column j at j*(m+1))
    double* cs = nullptr;       // [R][m]
    double* sn = nullptr;
    double* g = nullptr;        // [R][m+1]
    double* y = nullptr;        // [R][m]
    double* partial = nullptr;  // two banks of [R][nblk][m+2]
    double* hcol = nullptr;     // [R][m+2]
    double* bnorm = nullptr;    // [R]
    double* resid = nullptr;    // [R], followed by state
    double* tolv = nullptr;     // [R]
    double* nrm = nullptr;      // [R] norms handed to the host
    int32_t* state = nullptr;   // [R][4] right after resid: done flag, iterations, status, j
    int32_t* skip = nullptr;    // [R]
    int32_t* jcur = nullptr;    // Arnoldi step index read by replayed iteration graphs
    int32_t* Mr = nullptr;      // [R]
    size_t* voff = nullptr;     // [R]
    size_t* xoff = nullptr;     // [R]
    double* b = nullptr;        // pools: right-hand side, iterate, restart residual,
    double* x = nullptr;        // refinement residual and correction
    double* r = nullptr;
    double* rr = nullptr;
    double* d = nullptr;
    void* host_pinned = nullptr;
    std::vector<size_t> hvoff, hxoff;
    std::vector<void*> mem;
    // the operator step of an Arnoldi iteration, prepared once per restart length
    // and set of plan workspaces (op_key), with its argument tables in an arena of
    // its own; and that step with both Gram-Schmidt passes recorded as a graph
    std::shared_ptr<GroupedPass> op;
    std::vector<const void*> op_key;
    Arena op_arena;
    bool op_ran = false;       // has run eagerly: the tuned variants are settled
    // gexec[g] records 2^g Arnoldi steps of the current op (valid: all recorded)
    static constexpr int kGraphLevels = 4;
    bool graph_valid = false;
    hipGraphExec_t gexec[kGraphLevels] = {};
};
void free_krylov(KWork& k);

// Stage timing: a ring of event sets, one set per pass through the grid; each
// stage kernel records a start and a stop event in its own dispatch.
struct Timing {
    static constexpr int RING = 64;
    static constexpr int MAXST = 8;
    int enabled = 0;
    int events_made = 0;
    int ring_pos = 0, cur_set = -1;
    hipEvent_t ev[RING][2 * MAXST] = {};
    const char* set_names[RING][MAXST] = {};
    int set_used[RING] = {};
    const char* acc_names[16] = {};
    double acc_ms[16] = {};
    long long acc_n[16] = {};
    int n_acc = 0;
};
void timing_reset(Timing& t, int enable);
void timing_free(Timing& t);
// mean ms and call count per stage name since the last reset
int timing_read(Timing& t, double* ms, const char** names, int64_t* calls, int cap);

struct KrylovSet {
    std::vector<Inst> inst;
    int R = 0;
    KWork w;
    Arena* arena = nullptr;
};

}  // namespace ibdl

struct ibdl_plan_s {
    // description
    int dim = 2, n = 0, bc = 0, delta = 0, prec = 0, M = 0;
    int lap = IBDL_LAP_FD;  // Laplacian discretisation (ibdl_lap)
    int form = IBDL_FORM_DOUBLE_LAYER;  // ibdl_form
    double eta = 0.0;       // completed formulation: weight of the single layer
    double lo[3] = {0, 0, 0}, length = 1, h = 1, alpha = 0;
    int P = 0;          // complex elements per line of the tiled half spectrum (>= n/2+1)
    int W = 0;          // half-spectrum width n/2+1
    int nlines = 0;     // n^(dim-1) x-lines
    size_t spec_elems = 0;  // nlines * P
    int gpp = 0;        // gather partials per point: 4^(dim-1)

    // geometry in (key, index) order
    uint32_t* perm = nullptr;       // [M] caller index of sorted point s
    uint32_t* invperm = nullptr;    // [M] sorted position of caller point k
    uint32_t* key = nullptr;        // [M] key of caller point k
    uint32_t* skey = nullptr;       // [M] key of sorted point s
    int32_t* cell = nullptr;        // [M][3] cell of sorted point s
    double* taps64 = nullptr;       // [M][3][4] phi(p - t) for p = c-1..c+2, sorted order
    float* taps32 = nullptr;
    double* X = nullptr;            // [M][3] caller order (coordinates as given)
    double* nrm = nullptr;          // [M][3] caller order
    double* wgt = nullptr;          // [M] caller order
    int32_t* line_start = nullptr;  // [nlines+1] first sorted point of each x-line (cell key / n)

    ibdl::Csr dip, mono;

    // line/plane sets
    uint8_t* spread_line_mask = nullptr;   // [nlines]
    uint8_t* gather_line_mask = nullptr;   // [nlines]
    uint8_t* spread_plane_mask = nullptr;  // [n] (3-D)
    uint8_t* gather_plane_mask = nullptr;  // [n] (3-D)
    int32_t* spread_lines = nullptr;
    int32_t* gather_lines = nullptr;
    int32_t* spread_planes = nullptr;
    int32_t* gather_planes = nullptr;
    int n_spread_lines = 0, n_gather_lines = 0, n_spread_planes = 0, n_gather_planes = 0;

    // tables
    double* tw64 = nullptr;   // [n] exp(-2 pi i m/n) as (re, im)
    float* tw32 = nullptr;
    double* s2_64 = nullptr;  // [n] minus the 1-D Laplacian eigenvalue of mode m: (4/h^2) sin^2(pi m/n)
                              // (finite differences) or (2 pi k/L)^2, k the signed frequency (spectral)
    float* s2_32 = nullptr;
    // 2-D mixed plans: the FP32 column pass's factor norm / lambda(kx, ky) for every
    // element of the half spectrum, in its column-tile layout [tile][ky][C]
    float* sym32 = nullptr;

    // near-boundary step, allocated at its first use: unit strengths, the candidate
    // mask of the re-interpolation and two reference values of the indicator
    double* ones = nullptr;
    uint8_t* fix_mask = nullptr;
    double* fix_refs = nullptr;
    // completed formulation: Q2 with K Q2 = 1 and, last, eta w.Q2 (solved at the first solve)
    double* cq2 = nullptr;

    ibdl::Workspace ws;
    ibdl::KrylovSet ks;     // Krylov state of solves through this plan alone
    ibdl::Arena arena;

    // stage timing (the plan's own record, or one shared by the plans of a batch)
    ibdl::Timing own_timing;
    ibdl::Timing* tm = &own_timing;

    std::vector<void*> allocs;     // everything to free
    std::vector<void*> build_tmp;  // construction temporaries
    hipStream_t last_stream = nullptr;  // stream of the latest call
};

// Many independent instances solved together (one plan per instance).
struct ibdl_batch_s {
    hipStream_t last_stream = nullptr;
    std::vector<ibdl_plan> plans;
    ibdl::KrylovSet ks;
    ibdl::Arena arena;
    ibdl::Timing timing;
};

namespace ibdl {

// Inputs and outputs of one pass of L^-1 through the grid.
struct PipeIn {
    const double* q_dip = nullptr;   // [nrhs][M] dipole strengths (S~ q)
    double c_dip = 0;
    const double* q_mono = nullptr;  // [nrhs][M] monopole strengths (S q)
    double c_mono = 0;
    const double* grid = nullptr;    // [nrhs][n^dim] grid forcing
    double c_grid = 0;
    size_t q_stride = 0;             // distance between right-hand sides of q_dip/q_mono (0: M)
    size_t q_jstride = 0;            // added per iteration index (Krylov basis)
    const int32_t* skip = nullptr;   // per-rhs flags (stride 4): set -> the rhs is not processed
    // q_dip is first copied in the pass's precision into the plan's workspace in
    // groups of four right-hand sides (ws.qf), which the spread reads instead
    bool pack_q = false;
    // invert Lap_h with alpha = 0 (mean-zero) whatever the plan's alpha (FP64 passes)
    bool alpha_zero = false;
};
struct PipeOut {
    // gather: out[k] = cA * (S* u)_k + cB * in[k] + cC * in2[k]   (strides 0: M)
    double* out = nullptr;
    size_t out_stride = 0;
    size_t out_jstride = 0;          // added per iteration index
    double cA = 0;
    const double* in = nullptr;
    size_t in_stride = 0;
    size_t in_jstride = 0;
    double cB = 0;
    const double* in2 = nullptr;
    size_t in2_stride = 0;
    double cC = 0;
    // gather only: also the block partial sums of <out, V_i>, i < dots_nv + iteration index
    const double* dots_V = nullptr;
    size_t dots_vstride = 0;
    int dots_nv = 0;
    double* dots = nullptr;
    size_t dots_rhs = 0;
    int dots_stride = 0;
    // grid: u = the full grid field
    double* u = nullptr;
};

// records msg as this host thread's last error and returns status
ibdl_status set_error(int status, const std::string& msg);

// Device memory is stream ordered (the device's default memory pool, which keeps
// freed memory for reuse): allocations and frees are placed on the calling
// thread's current allocation stream, set by AllocStream for the duration of a call.
void* dev_alloc(std::vector<void*>& owner, size_t bytes);
void* dev_alloc(ibdl_plan p, size_t bytes);
void dev_free(void* ptr);
hipStream_t alloc_stream();
struct AllocStream {
    hipStream_t prev;
    explicit AllocStream(hipStream_t s);
    ~AllocStream();
};
// Pinned host staging blocks, kept for reuse until the process ends (releasing
// pinned memory can wait for the whole device).
void* pinned_get(size_t bytes);
void pinned_put(void* ptr);
void ensure_workspace(ibdl_plan p, int nrhs);

// One job of a grid pass: a plan, its right-hand sides, inputs and outputs.
struct PassJob {
    ibdl_plan p;
    int nrhs;
    PipeIn in;
    PipeOut out;
};
// A grid pass prepared for one or more jobs of the same dimension, grid size and
// precision; run() launches every stage once for all jobs.
struct PreparedPass {
    virtual ~PreparedPass() {}
    virtual void upload(Arena& arena, hipStream_t st) = 0;  // several jobs only; stages, caller flushes
    virtual void run(int it, hipStream_t st) = 0;            // it: iteration index
    // the same with the iteration index *itp + off, *itp read on the device
    void run_dev(const int32_t* itp, int off, hipStream_t st) {
        itp_ = itp;
        run(off, st);
        itp_ = nullptr;
    }

protected:
    const int32_t* itp_ = nullptr;
};

// A grid pass over chosen instances of a set, one prepared pass per
// (dimension, grid size, precision) group.
struct GroupedPass {
    std::vector<std::unique_ptr<PreparedPass>> parts;
    void run(int it, hipStream_t st) {
        for (auto& p : parts) p->run(it, st);
    }
    void run_dev(const int32_t* itp, int off, hipStream_t st) {
        for (auto& p : parts) p->run_dev(itp, off, st);
    }
};
std::unique_ptr<PreparedPass> prepare_f64(const std::vector<PassJob>& jobs);
std::unique_ptr<PreparedPass> prepare_f32(const std::vector<PassJob>& jobs);
// fp64 forces the FP64 pipeline on a mixed plan (right-hand sides, residuals, grid solutions)
std::unique_ptr<PreparedPass> prepare_pass(const std::vector<PassJob>& jobs, bool fp64);
void run_pipeline(ibdl_plan p, int nrhs, const PipeIn& in, const PipeOut& out, hipStream_t st,
                  bool fp64 = false);
int tile_pitch_f64(int n);
int tile_pitch_f32(int n);
int col_width_f64(int n);
int col_width_f32(int n);
// column rows per workgroup of the 3-D symbol pass (the K of k_col)
int z_rows_f64(int n);
int z_rows_f32(int n);
void build_plan(ibdl_plan p, const ibdl_desc* d, hipStream_t st);
// near-boundary step (nearfix.hip): App. D indicator and flags, App. A fix-up
void nearfix_indicator(ibdl_plan p, double* chi, uint8_t* flags, hipStream_t st);
// completed formulation (forms.hip): vectors z = [Q; ubar] of M + 1 values per rhs
void completed_apply(ibdl_plan p, int nrhs, const double* z, double* out, hipStream_t st);
void completed_rhs(ibdl_plan p, int nrhs, const double* data, const double* g, double* b, hipStream_t st);
void completed_eval_grid(ibdl_plan p, int nrhs, const double* z, const double* g, double* u, hipStream_t st);
int completed_solve(ibdl_plan p, int nrhs, const double* data, const double* g, const ibdl_solve_opts& o,
                    double* sol, double* u, ibdl_solve_info* info, hipStream_t st);
// single-layer (IB constraint) formulation with MINRES (forms.hip)
void ibsl_apply(ibdl_plan p, int nrhs, const double* q, double* out, hipStream_t st);
void ibsl_eval_grid(ibdl_plan p, int nrhs, const double* f, const double* g, double* u, hipStream_t st);
int ibsl_solve(ibdl_plan p, int nrhs, const double* data, const double* g, const ibdl_solve_opts& o, double* sol,
               double* u, ibdl_solve_info* info, hipStream_t st);
void nearfix_fixup(ibdl_plan p, int nrhs, const double* u, const double* ub, const uint8_t* flags, double m1,
                   double m2, double* uout, hipStream_t st);
void free_build_tmp(ibdl_plan p);
// frees every device allocation of a plan in stream order on st (no wait) and the plan
void release_plan(ibdl_plan p, hipStream_t st);
// GMRES (with FP64 refinement for mixed plans) for every instance of the set:
// per instance i the data, forcing (or null), initial iterate (or null) and
// solution buffers, [nrhs_i][M_i] / [nrhs_i][n^d].  info: host [R].
void solve_set(KrylovSet& ks, const std::vector<const double*>& data, const std::vector<const double*>& g,
               const std::vector<const double*>& x0, const ibdl_solve_opts& o, const std::vector<double*>& sol,
               ibdl_solve_info* info, hipStream_t st, int* overall, const std::vector<double*>& u = {});

// Tile autotuner: per pass configuration, the row-block variant measured fastest.
// dense: output mode (0 points, 1 grid, 2 both); grid_in: the forward row stage
// reads a forcing grid (every line) rather than the spread lines alone
struct TuneKey {
    int rbytes, dim, n, stage, dense, minr, totr, multi, grid_in;
    bool operator<(const TuneKey& o) const {
        const int a[9] = {rbytes, dim, n, stage, dense, minr, totr, multi, grid_in};
        const int b[9] = {o.rbytes, o.dim, o.n, o.stage, o.dense, o.minr, o.totr, o.multi, o.grid_in};
        for (int i = 0; i < 9; ++i)
            if (a[i] != b[i]) return a[i] < b[i];
        return false;
    }
};
inline int tune_bucket(int v) {  // 1, 2-3, 4-7, ... -> 0, 1, 2, ...
    int b = 0;
    while ((2 << b) <= v) ++b;
    return b;
}
int tune_lookup(const TuneKey& k);                      // variant or -1
void tune_store(const TuneKey& k, int variant, float ms);
bool tune_enabled();
int tune_forced();                                       // row variant forced for tests, or -1
// set while this thread records a graph: untuned stages take the heuristic
// variant instead of timing the others
bool& capturing();
bool graphs_enabled();
void note_graphs(int64_t recorded, int64_t replays);

// timing helpers used by the pipeline: events to pass to the stage's launch
// (both null when timing is off); stage 0 opens a new event set
struct StageEv {
    hipEvent_t a = nullptr, b = nullptr;
};
StageEv stage_events(ibdl_plan p, int idx, const char* name);

}  // namespace ibdl
