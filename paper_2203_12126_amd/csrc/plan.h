// Internal plan structure of the IBDL library (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
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
    double* w64 = nullptr;          // [nnz] weight
    float* w32 = nullptr;           // [nnz] weight rounded to FP32
    int32_t* line_act = nullptr;    // [nlines+1] first active node of each x-line
};

struct Workspace {
    int cap_rhs = 0;
    void* spec = nullptr;       // [cap][nlines*P] complex
    void* part = nullptr;       // [cap][M][4^(dim-1)] gather partial sums
};

struct Krylov {
    int cap_rhs = 0, cap_m = 0, nblk = 0;
    double* V = nullptr;        // [rhs][m+1][M]
    double* H = nullptr;        // [rhs][m+1][m]  (column-major by j: H[j*(m+1) + i])
    double* cs = nullptr;       // [rhs][m]
    double* sn = nullptr;       // [rhs][m]
    double* g = nullptr;        // [rhs][m+1]
    double* y = nullptr;        // [rhs][m]
    double* partial = nullptr;  // [rhs][nblk][m+2]
    double* hcol = nullptr;     // [rhs][m+2]
    double* bnorm = nullptr;    // [rhs]
    double* resid = nullptr;    // [rhs]
    double* tolv = nullptr;     // [rhs]
    int32_t* state = nullptr;   // [rhs][4]: done flag, iterations, status, j
    int32_t* skip = nullptr;    // [rhs]
    double* b = nullptr;        // [rhs][M] right-hand side
    double* r = nullptr;        // [rhs][M] restart residual
    double* rr = nullptr;       // [rhs][M] refinement residual
    double* d = nullptr;        // [rhs][M] refinement correction
    void* host_pinned = nullptr;
};

struct JobRing {
    char* host = nullptr;
    char* dev = nullptr;
    size_t cap = 0, pos = 0;
    std::vector<void*>* owner = nullptr;
};

}  // namespace ibdl

struct ibdl_plan_s {
    // description
    int dim = 2, n = 0, bc = 0, delta = 0, prec = 0, M = 0;
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
    double* s2_64 = nullptr;  // [n] (4/h^2) sin^2(pi m/n)
    float* s2_32 = nullptr;

    ibdl::Workspace ws;
    ibdl::Krylov kr;

    // stage timing: a ring of event sets, one set per pass through the grid; each
    // stage kernel records a start and a stop event in its own dispatch
    static constexpr int RING = 64;
    static constexpr int MAXST = 8;
    int timing = 0;
    int events_made = 0;
    int ring_pos = 0, cur_set = -1;
    hipEvent_t ev[RING][2 * MAXST] = {};
    const char* set_names[RING][MAXST] = {};
    int set_used[RING] = {};
    const char* acc_names[16] = {};
    double acc_ms[16] = {};
    long long acc_n[16] = {};
    int n_acc = 0;

    std::vector<void*> allocs;  // everything to free
    ibdl::JobRing ring;
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

void* dev_alloc(std::vector<void*>& owner, size_t bytes);
void* dev_alloc(ibdl_plan p, size_t bytes);
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
    virtual void upload(JobRing& ring, hipStream_t st) = 0;  // only needed for several jobs
    virtual void run(int it, hipStream_t st) = 0;            // it: iteration index
};
std::unique_ptr<PreparedPass> prepare_f64(const std::vector<PassJob>& jobs);
std::unique_ptr<PreparedPass> prepare_f32(const std::vector<PassJob>& jobs);
// fp64 forces the FP64 pipeline on a mixed plan (right-hand sides, residuals, grid solutions)
std::unique_ptr<PreparedPass> prepare_pass(const std::vector<PassJob>& jobs, bool fp64);
void run_pipeline(ibdl_plan p, int nrhs, const PipeIn& in, const PipeOut& out, hipStream_t st,
                  bool fp64 = false);
// staging area for argument tables: pinned host copy, device copy, wraps after a stream sync
void* ring_put(JobRing& r, const void* src, size_t bytes, hipStream_t st);
int tile_pitch_f64(int n);
int tile_pitch_f32(int n);
void build_plan(ibdl_plan p, const ibdl_desc* d, hipStream_t st);
void gmres_solve(ibdl_plan p, int nrhs, const double* data, const double* g, const ibdl_solve_opts& o,
                 double* sol, ibdl_solve_info* info, hipStream_t st, int* overall);

// timing helpers used by the pipeline: events to pass to the stage's launch
// (both null when timing is off); stage 0 opens a new event set
struct StageEv {
    hipEvent_t a = nullptr, b = nullptr;
};
StageEv stage_events(ibdl_plan p, int idx, const char* name);

}  // namespace ibdl
