// A solve of a Krylov set (one or more plans with their right-hand sides) as a
// resumable sequence of device work: the right-hand side, restarted GMRES, FP64
// refinement of mixed plans, optional true residuals, the solution copy-out and
// optionally the grid solution.  advance() does the host logic for the last
// wait point and enqueues the work up to the next one; ready() polls that wait
// point without blocking, so a scheduler can interleave many tasks on their own
// streams.
#pragma once
#include <functional>
#include <memory>
#include <vector>

#include "plan.h"

namespace ibdl {

// per-instance device buffers of a solve
struct SolveIO {
    std::vector<const double*> data, g, x0;   // x0 entries may be null
    std::vector<double*> sol;
    std::vector<double*> u;                   // grid solutions (empty or null entries: none)
    std::vector<const double*> vb;            // Neumann V_b for the grid solution
};

// A grid pass over chosen instances of a set, one prepared pass per
// (dimension, grid size, precision) group.
using JobMaker = std::function<PassJob(size_t)>;
// tables go to the set's arena, or to *ar when given
GroupedPass prepare_grouped(KrylovSet& ks, const std::vector<size_t>& which, const JobMaker& make, bool fp64,
                            hipStream_t st, Arena* ar = nullptr);

class SolveTask {
public:
    // graphs: the Arnoldi steps may be replayed from a recorded graph (also subject
    // to the process-wide switch and to stage timing being off)
    SolveTask(KrylovSet& ks, SolveIO io, const ibdl_solve_opts& o, hipStream_t st, bool graphs = true);
    ~SolveTask();
    bool done() const { return phase_ == DONE; }
    bool ready();          // the last wait point has been reached (non-blocking)
    void wait();           // block until it has
    void advance();        // requires ready(); enqueues the next stretch of work
    void run_to_end();     // wait/advance until done
    // per-rhs results (host [R]) and the worst status
    void results(ibdl_solve_info* info, int* overall) const;
    int total_iters() const;

private:
    enum Phase { BEGIN, ITER, KEND, OUT, DONE };
    void mark();                                  // record the wait point
    void kstart(const double* b, double* x, bool x_zero);
    void enqueue_iters(int j0, int c);
    void prepare_op();                            // the set's Arnoldi operator step, current
    bool capture_steps(int g);  // record 2^g Arnoldi steps as one graph
    void enqueue_chunk(int c);
    void snapshot(int buf);
    void after_krylov();
    void collect();
    void finish_mixed();
    void output();
    void residual(const double* b, const double* x, double* r, bool fp64, bool with_grid = false);
    bool grid_fusable(size_t i) const;
    void norms_async(const double* pool, double* host);

    KrylovSet& ks_;
    SolveIO io_;
    ibdl_solve_opts o_;
    hipStream_t st_;
    hipEvent_t ev_ = nullptr;
    Phase phase_ = BEGIN;
    int m_ = 0, R_ = 0;
    // current Krylov run
    const double* kb_ = nullptr;
    double* kx_ = nullptr;
    int kmaxit_ = 0, ktotal_ = 0, kj_ = 0;
    int snap_buf_ = 0;      // staging buffer of the last snapshot
    int snap_iter_ = 0;     // cycle steps enqueued before it
    int queued_after_ = 0;  // steps enqueued after it
    int prev_iter_ = -1;    // cycle steps before the previous snapshot (-1: none this cycle)
    std::vector<double> prev_;
    // Arnoldi steps replayed from the set's recorded graph once the operator step
    // has run eagerly (which settles the tuned variants); the step index then lives
    // on the device: dev_j_ is its value after the queued work (-1: not known)
    bool use_graph_ = false, graph_unmarked_ = false;
    int dev_j_ = -1;
    // solve state
    bool any_mixed_ = false, refining_ = false, fill_true_ = false;
    int round_ = 0;
    std::vector<double> bn_, tol_, est_, truer_;
    std::vector<int> skip_, iters_, status_, fp64_;
    std::vector<int> budget_;  // Arnoldi steps each rhs may still take (maxit less its own)
    std::vector<char> grid_done_;  // per instance: u written by the last residual pass
};

}  // namespace ibdl
