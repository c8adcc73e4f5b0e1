/*
 * ibdl.h -- C ABI of the MI355X (gfx950) IBDL hot path.
 *
 * The Immersed Boundary Double Layer method (Leathers & Guy) solves
 *     Lap u - alpha u = g in Omega,   u = U_b (Dirichlet) or du/dn = V_b (Neumann) on Gamma
 * on a periodic box by representing u with a regularised double layer (dipole
 * spread) of strength Q on the boundary points.  Its hot path is the matrix-free
 * boundary operator applied at every GMRES iteration:
 *     Dirichlet:  A q = -S* L^-1 S~ q + q/2      (Sec. 5.3: the equation for Q once L is inverted)
 *     Neumann:    A q = -S* L^-1 S~ q - q/2      (Sec. 4.4: the equation for the unknown U_b)
 * with S~ q = div(S (q n)) the dipole spread (Sec. 5.2), S the discrete spread and
 * S* the discrete interpolation (Sec. 5.2), delta_h the product of Peskin's
 * four-point kernel phi over the axes (Sec. 5.2) and L = Lap_h - alpha the periodic
 * 5-point (2-D) / 7-point (3-D) operator (Sec. 5.1).
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers (for example a torch tensor's
 *    data_ptr on the current GPU) unless the comment says "host".
 *  - Arrays are dense, C-ordered, FP64.  Boundary arrays are indexed in the
 *    caller's point order.  Grid arrays are [iz][iy][ix] with x fastest; node
 *    (ix,iy,iz) sits at lo + h*(ix,iy,iz), h = length/n.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Work is enqueued on it; "async" entry points return before it finishes.
 *  - The caller owns every input and output buffer.  A plan owns its device
 *    workspace and a sorted copy of the geometry; the geometry the caller passed
 *    may be freed once ibdl_plan_create returns.
 *  - Arguments are validated before anything is written.  On failure the
 *    status is returned and ibdl_last_error() (thread-local) describes it.
 *  - A plan is not thread-safe: use it from one host thread and one stream at a
 *    time.  No C++ exception crosses this interface.
 */
#ifndef IBDL_H
#define IBDL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibdl_plan_s* ibdl_plan;
typedef struct ibdl_batch_s* ibdl_batch;
typedef struct ibdl_server_s* ibdl_server;

typedef enum {
    IBDL_OK = 0,
    IBDL_ERR_ARG = 1,      /* invalid argument (sizes, pointers, enum values)      */
    IBDL_ERR_OOM = 2,      /* device allocation failed                              */
    IBDL_ERR_HIP = 3,      /* a HIP runtime call failed                             */
    IBDL_ERR_NOCONV = 4,   /* GMRES stopped at maxit above tol (best iterate written) */
    IBDL_ERR_NUMERIC = 5,  /* non-finite input or residual                          */
    IBDL_ERR_STATE = 6     /* wrong state (e.g. request still pending)              */
} ibdl_status;

typedef enum { IBDL_DIRICHLET = 0, IBDL_NEUMANN = 1 } ibdl_bc;

/* Discrete delta kernel phi (delta_h(x) = prod_d phi(x_d/h)/h):
 * PESKIN4 is the paper's kernel (Sec. 5.2);
 * COSINE4 is phi(r) = (1 + cos(pi r/2))/4 for |r| < 2. */
typedef enum { IBDL_DELTA_PESKIN4 = 0, IBDL_DELTA_COSINE4 = 1 } ibdl_delta;

/* FP64: spread, FFT solve and interpolation in FP64.
 * MIXED: spread (compensated sums), FFT solve and interpolation in FP32; the
 *        identity term, all GMRES arithmetic and every output stay FP64. */
typedef enum { IBDL_PREC_FP64 = 0, IBDL_PREC_MIXED = 1 } ibdl_prec;

/* Discretisation of the Laplacian in L = Lap_h - alpha (both diagonal in the DFT):
 * FD is the 5-point (2-D) / 7-point (3-D) stencil, eigenvalues
 * -(4/h^2) sin^2(pi m_d/n) per axis (Sec. 5.1); SPECTRAL is the Fourier-spectral
 * Laplacian, -(2 pi k_d/L)^2 per axis with k_d the signed frequency of mode m_d
 * (Sec. 6.2.1).  The divergence inside S~ stays the centred difference of Sec. 5.2
 * in both. */
typedef enum { IBDL_LAP_FD = 0, IBDL_LAP_SPECTRAL = 1 } ibdl_lap;

/* Formulation of the boundary equation.
 * DOUBLE_LAYER: the IBDL system (Sec. 4.1, Sec. 4.4, Sec. 5.3), Dirichlet or Neumann.
 * COMPLETED: the completed IBDL system for the Poisson equation (Sec. 5.4.1,
 *   App. C): alpha = 0, Dirichlet, eta > 0.  Its unknown is z = [Q; ubar]
 *   (M + 1 values per right-hand side) and its operator the bordered matrix
 *     [-S* D0^-1 (S~ + eta S) + I/2,  1;  eta w^T,  0]
 *   (D0^-1 the mean-zero inverse of the periodic Laplacian, w the point weights),
 *   with right-hand side [U_b - S* D0^-1 g~;  h^d sum_x g~(x)] and grid solution
 *   u = D0^-1 (g~ - (S~ + eta S) Q) + ubar.  For such plans q, Aq, b and sol of
 *   ibdl_apply / ibdl_rhs / ibdl_solve / ibdl_solve_grid / ibdl_eval_grid hold
 *   M + 1 values per right-hand side ([nrhs][M+1], ubar last); the boundary
 *   data stay [nrhs][M].  Not accepted by batches and servers. */
/* SINGLE_LAYER: the IB constraint system the paper compares against (Sec. 2.1;
 *   Tables 1 and 2): Dirichlet, FP64.  ibdl_apply gives -(S* L^-1 S) F, ibdl_rhs
 *   U_b - S* L^-1 g~, ibdl_eval_grid u = L^-1 (g~ - S F), and ibdl_solve runs
 *   MINRES on the device in the inner product <x, y>_W = sum_k w_k x_k y_k, in
 *   which the operator is self-adjoint (plain MINRES for equal weights), from
 *   F = 0 until the W-norm residual estimate falls to tol; info.iters counts
 *   operator applications and rel_resid_est is that estimate.  opts->restart is
 *   ignored.  Not accepted by batches and servers. */
typedef enum { IBDL_FORM_DOUBLE_LAYER = 0, IBDL_FORM_COMPLETED = 1, IBDL_FORM_SINGLE_LAYER = 2 } ibdl_form;

typedef struct {
    int32_t dim;          /* 2 or 3                                                        */
    int32_t n;            /* nodes per axis, n = 2^a 3^b, 8 <= n <= 2048 (2-D), <= 512 (3-D) */
    double lo[3];         /* box origin (entries beyond dim ignored)                        */
    double length;        /* periodic box side L > 0 (Sec. 5.1: dx = L/n)                   */
    double alpha;         /* L = Lap_h - alpha, alpha >= 0 (alpha = k^2); 0 -> mean-zero inverse */
    int32_t bc;           /* ibdl_bc                                                        */
    int32_t delta;        /* ibdl_delta                                                     */
    int32_t prec;         /* ibdl_prec                                                      */
    int32_t npts;         /* M >= 1 boundary points; M < 2^28 / 32 (2-D), 2^28 / 160 (3-D)  */
    const double* X;      /* device [M][dim] point coordinates (any real values, wrapped periodically) */
    const double* normal; /* device [M][dim] unit normals pointing OUT of Omega (Sec. 4.1)    */
    const double* weight; /* device [M] quadrature weights: arclength Delta s_i (2-D, Sec. 5.2)
                             or area dA_i (3-D, Sec. 6.7), > 0                               */
    int32_t lap;          /* ibdl_lap                                                       */
    int32_t form;         /* ibdl_form                                                      */
    double eta;           /* COMPLETED: weight eta > 0 of the single layer (the paper uses 10) */
} ibdl_desc;

typedef struct {
    double tol;           /* stop when ||b - A x||_2 <= tol ||b||_2 (Arnoldi estimate), Sec. 5.3 */
    int32_t restart;      /* Krylov subspace size before restart, 1..200                    */
    int32_t maxit;        /* maximum operator applications in the Krylov loop               */
    const double* x0;     /* device [nrhs][M] initial guess, or NULL for x0 = 0 (the paper's) */
    int32_t true_residual;/* 1: spend one more apply per rhs to report ||b - A x||/||b||     */
} ibdl_solve_opts;

typedef struct {
    int32_t iters;          /* operator applications in the Krylov loop                     */
    double rel_resid_est;   /* Arnoldi residual estimate / ||b||                            */
    double rel_resid_true;  /* ||b - A x|| / ||b|| if requested, else -1                    */
    int32_t status;         /* ibdl_status of this right-hand side                          */
    int32_t fp64_applies;   /* FP64 operator passes spent on residuals (mixed refinement)    */
} ibdl_solve_info;

/* Build a plan for one geometry (Sec. 5.1-5.2): cell binning of the points by the
 * integer key  key = row-major index of floor((X - lo)/h) mod n  (x fastest, IEEE FP64),
 * a stable sort of (key, point index), the per-point delta taps, the sparse dipole
 * spread (and, for Neumann, monopole spread) structure, FFT twiddles and the symbol
 * of L.  Copies the geometry; synchronises `stream` before returning.
 * Errors: IBDL_ERR_ARG (bad desc), IBDL_ERR_NUMERIC (non-finite X/normal/weight),
 * IBDL_ERR_OOM, IBDL_ERR_HIP.  *out is set only on success. */
ibdl_status ibdl_plan_create(const ibdl_desc* desc, void* stream, ibdl_plan* out);

/* Free a plan and its device workspace (waits for work queued on the plan's last stream). */
ibdl_status ibdl_plan_destroy(ibdl_plan plan);

/* Host-only estimate of the device bytes a plan plus solve workspace for `nrhs`
 * right-hand sides and Krylov size `restart` occupies (used for admission): an
 * upper bound, rounded up to whole 2 MiB device pages plus one.  Returns 0 for
 * an invalid desc. */
size_t ibdl_plan_footprint(const ibdl_desc* desc, int32_t nrhs, int32_t restart);

/* Aq[r] = A q[r] for r < nrhs (async).  q, Aq: device [nrhs][M], must not overlap.
 * A is the Dirichlet or Neumann operator chosen by the plan's bc. */
ibdl_status ibdl_apply(ibdl_plan plan, int32_t nrhs, const double* q, double* Aq, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): ibdl_apply with the
 * pass's half spectra and gather partial sums in a fixed device scratch area of
 * 256 MiB that the library holds on each device from its first call there until
 * the process ends.  Calls no hipMalloc, hipFree or other allocating routine; row
 * shapes not tuned yet take the fixed rule instead of being timed.  The scratch
 * must hold nrhs * (spectrum + partials) of the plan's precision: FP64 plans
 * nrhs * (nlines * pitch * 16 + M * 4^(dim-1) * 8) bytes, MIXED plans half of it
 * (ibdl_plan_get_stats gives nlines and pitch); larger calls return IBDL_ERR_ARG
 * before any work.  Every call on a device shares that device's scratch, so calls
 * whose work overlaps on one device (different streams, or host threads) race:
 * order them on one stream.  Results equal ibdl_apply's. */
ibdl_status ibdl_apply_noalloc(ibdl_plan plan, int32_t nrhs, const double* q, double* Aq, void* stream);

/* Right-hand side of the boundary equation (async):
 *   Dirichlet  b = U_b - S* L^-1 g~               (Sec. 5.3, right side of the equation for Q)
 *   Neumann    b = S* L^-1 (S V_b - g~)           (Sec. 4.4, right side of the equation for U_b)
 * data: device [nrhs][M] U_b or V_b;  g: device [nrhs][n^dim] g~ or NULL (zero);
 * b: device [nrhs][M]. */
ibdl_status ibdl_rhs(ibdl_plan plan, int32_t nrhs, const double* data, const double* g,
                     double* b, void* stream);

/* Step 1 of the method (Sec. 4.2, Sec. 5.3): form the right-hand side and run
 * unpreconditioned restarted GMRES on the device (FP64 Arnoldi with classical
 * Gram-Schmidt applied twice, Givens rotations) for each right-hand side.
 * The right-hand side is formed in FP64 for every plan.  MIXED plans iterate
 * with the FP32-grid operator and refine: r = b - A x with the FP64 operator,
 * a further FP32-operator GMRES solve of A d = r, x += d, until the FP64
 * residual meets tol (at most 5 rounds); rel_resid_true is that FP64 residual.
 * sol: device [nrhs][M] receives Q (Dirichlet) or U_b (Neumann).
 * info: HOST [nrhs].  opts may be NULL (tol 1e-8, restart 50, maxit 500).
 * Blocks until done.  Returns IBDL_ERR_NOCONV if any rhs missed tol (its best
 * iterate is still written) and IBDL_ERR_NUMERIC on a non-finite residual. */
ibdl_status ibdl_solve(ibdl_plan plan, int32_t nrhs, const double* data, const double* g,
                       const ibdl_solve_opts* opts, double* sol, ibdl_solve_info* info,
                       void* stream);

/* Steps 1 and 2 in one call: ibdl_solve, then u = the grid solution of the
 * solution as ibdl_eval_grid gives it, with V_b = data for Neumann plans.  For
 * MIXED plans u comes out of the FP64 residual pass of the final iterate (one
 * pass gives u = L^-1 (g~ - S~ x [- S V_b]) on the grid and the residual
 * U_b - x/2 - S* u (Dirichlet) or x/2 - S* u (Neumann) at the points), so no
 * separate grid pass runs; u equals ibdl_eval_grid of the returned sol.
 * u: device [nrhs][n^dim]; the rest as for ibdl_solve. */
ibdl_status ibdl_solve_grid(ibdl_plan plan, int32_t nrhs, const double* data, const double* g,
                            const ibdl_solve_opts* opts, double* sol, double* u, ibdl_solve_info* info,
                            void* stream);

/* Step 2 of the method: the grid solution (async).
 *   Dirichlet  u = L^-1 (g~ - S~ Q)               (Sec. 4.2, step 2)
 *   Neumann    u = L^-1 (g~ - S~ U_b - S V_b)     (Sec. 4.4, the grid equation of the Neumann system)
 * sol: device [nrhs][M] (Q or U_b); vb: device [nrhs][M] V_b (Neumann only, else NULL);
 * g: device [nrhs][n^dim] or NULL; u: device [nrhs][n^dim]. */
ibdl_status ibdl_eval_grid(ibdl_plan plan, int32_t nrhs, const double* sol, const double* vb,
                           const double* g, double* u, void* stream);

/* Step 3 of the method (Sec. 4.2, Sec. 5.5), first part: the PDE domain on the
 * grid from the regularised indicator function of App. D (async).
 *   chi = -Delta_0^-1 S~ 1 - (its value at the corner node lo)
 * (the FP64 grid pipeline with unit strengths and the mean-zero inverse of the
 * Laplacian, whatever the plan's alpha).  For normals pointing away from the
 * region the boundary encloses (Omega that region) chi is about 1 in Omega and 0
 * elsewhere and flags = chi > 1/2; for normals pointing into it (Omega the rest of
 * the box) chi is about -1 inside and flags = chi > -1/2.  The orientation is the
 * sign of sum_k w_k (X_k - X_0) . n_k.  chi: device [n^dim] FP64 out; flags:
 * device [n^dim] uint8 out, 1 for nodes of Omega. */
ibdl_status ibdl_indicator(ibdl_plan plan, double* chi, uint8_t* flags, void* stream);

/* Step 3, second part: the re-interpolation of App. A (async).  u_out = u except at
 * nodes with flags = 1 whose nearest boundary point lies within m1 meshwidths:
 *   u(x_p) = u(x_A) |x_B - x_p| / |x_B - x_A| + u(x_B) |x_A - x_p| / |x_B - x_A|,
 * with x_A the point nearest x_p on the chord of its two nearest boundary points
 * (2-D; when the foot of the perpendicular leaves the chord, the two of its three
 * nearest points farthest apart span the chord, clamped to it), u(x_A) the linear
 * interpolation of ub along the chord; in 3-D x_A is the nearest boundary point and
 * u(x_A) its ub; x_B = x_A + (x_p - x_A)/|x_p - x_A| m2 h and u(x_B) the bilinear
 * (2-D) or trilinear (3-D) interpolation of u.  Values are read from u only.
 * The paper's widths are m1 = 6, m2 = 8 with the finite-difference Laplacian
 * (Sec. 6.1) and m1 = 2(log2 n - 4), m2 = m1 + 2 with the spectral one (Sec. 6.2.1).
 * u, u_out: device [nrhs][n^dim], distinct; ub: device [nrhs][M] boundary values
 * (U_b: the Dirichlet data, or the solved U_b of a Neumann plan), caller order;
 * flags: device [n^dim] from ibdl_indicator (or the caller's).  2-D points more
 * than two meshwidths apart may make the second and third nearest points fall
 * outside the cells searched (m1 + 5 cells around the node).
 * Errors: IBDL_ERR_ARG for 0 < m1 < m2 <= n/4 violated or missing buffers. */
ibdl_status ibdl_fixup(ibdl_plan plan, int32_t nrhs, const double* u, const double* ub, const uint8_t* flags,
                       double m1, double m2, double* u_out, void* stream);

/* The plan's binning (for inspection and tests), copied to HOST arrays of M
 * entries: key[k] = cell key of caller point k; perm[s] = caller index of the
 * s-th point in (key, index) order.  Either pointer may be NULL. */
ibdl_status ibdl_plan_binning(ibdl_plan plan, uint32_t* key_host, uint32_t* perm_host);

/* Per-stage device timing.  While enabled, every pass of the plan through the
 * grid (apply, rhs, solve iterations, eval_grid) records HIP events on its
 * stream before each stage and at its end; enabling (again) clears the record.
 * ibdl_plan_stage_times waits for the recorded events and returns, per stage
 * name, the mean time in milliseconds (ms_host) and the number of timed calls
 * (calls); names receives static strings.  Up to `cap` stages are written and
 * *count receives the number of distinct stages.  Any output pointer may be NULL. */
ibdl_status ibdl_plan_set_timing(ibdl_plan plan, int32_t enable);
ibdl_status ibdl_plan_stage_times(ibdl_plan plan, double* ms_host, const char** names,
                                  int64_t* calls, int32_t cap, int32_t* count);

/* Sizes of a plan's data structures (for byte accounting and inspection). */
typedef struct {
    int32_t nlines;            /* x-lines of the grid, n^(dim-1)                          */
    int32_t pitch;             /* complex elements per half-spectrum row (>= n/2+1)        */
    int32_t n_spread_lines;    /* x-lines that receive dipole forcing                      */
    int32_t n_gather_lines;    /* x-lines some boundary point interpolates from            */
    int32_t n_spread_planes;   /* 3-D: z-planes holding spread lines (else 0)              */
    int32_t n_gather_planes;   /* 3-D: z-planes holding gather lines (else 0)              */
    int32_t dip_active_nodes;  /* grid nodes reached by the dipole spread                  */
    int64_t dip_nnz;           /* (node, point) entries of the dipole spread               */
    int64_t mono_nnz;          /* entries of the monopole spread (Neumann plans, else 0)   */
    int32_t col_tile;          /* columns per tile of the half spectrum, in the precision
                                  of the plan's Arnoldi operator (FP32 for MIXED)          */
    int32_t z_rows;            /* 3-D: z-columns per workgroup of the symbol pass in that
                                  precision (k_col's K); 2-D: 1                             */
} ibdl_plan_stats;

ibdl_status ibdl_plan_get_stats(ibdl_plan plan, ibdl_plan_stats* out_host);

/* ---------------------------------------------------------------------------
 * Batches: many independent problems (each its own geometry, grid size, alpha,
 * boundary condition, precision and number of right-hand sides) carried through
 * the method together.  Every grid pass launches each stage once per group of
 * instances with the same dimension, grid size and precision (a per-instance
 * argument table maps each workgroup to its instance), and every GMRES kernel
 * launches once over all right-hand sides of the batch.  The arithmetic of an
 * instance is the same as in a solve through its own plan: results are
 * bit-identical to ibdl_solve / ibdl_apply / ibdl_eval_grid on that instance.
 * Per-instance array arguments are HOST arrays of `count` DEVICE pointers, each
 * laid out as for the single-plan entry point ([nrhs_i][M_i] or [nrhs_i][n_i^dim]).
 * A batch is not thread-safe; its entry points wait for work already queued on
 * `stream` before they start.
 * ------------------------------------------------------------------------- */

/* Build one plan per instance (as ibdl_plan_create) and the batch's workspace.
 * descs: host [count]; nrhs: host [count], each >= 1.  Synchronises `stream`.
 * Errors: IBDL_ERR_ARG (the message names the first bad instance), IBDL_ERR_NUMERIC,
 * IBDL_ERR_OOM, IBDL_ERR_HIP.  *out is set only on success. */
ibdl_status ibdl_batch_create(const ibdl_desc* descs, int32_t count, const int32_t* nrhs, void* stream,
                              ibdl_batch* out);

/* Free the batch, its plans and workspace (waits for the device). */
ibdl_status ibdl_batch_destroy(ibdl_batch batch);

/* Number of instances and of right-hand sides over all instances (either may be NULL). */
ibdl_status ibdl_batch_size(ibdl_batch batch, int32_t* count, int32_t* total_rhs);

/* ibdl_plan_get_stats of instance i (0 <= i < count). */
ibdl_status ibdl_batch_get_stats(ibdl_batch batch, int32_t i, ibdl_plan_stats* out_host);

/* Aq_i = A_i q_i for every instance (Sec. 5.3 / Sec. 4.4 operators; async after the wait). */
ibdl_status ibdl_batch_apply(ibdl_batch batch, const double* const* q, double* const* Aq, void* stream);

/* ibdl_solve for every instance (Sec. 4.2, Sec. 5.3): right-hand sides, GMRES
 * with the instances' own stopping tests, FP64 refinement of MIXED instances.
 * data, sol: per instance; g: NULL (no forcing anywhere) or per instance with
 * NULL entries allowed.  opts as for ibdl_solve except that opts->x0 must be NULL.
 * info: HOST [total_rhs] in instance order.  Blocks until done.  Returns
 * IBDL_ERR_NOCONV / IBDL_ERR_NUMERIC if any right-hand side ended so (every
 * other solution is still written). */
ibdl_status ibdl_batch_solve(ibdl_batch batch, const double* const* data, const double* const* g,
                             const ibdl_solve_opts* opts, double* const* sol, ibdl_solve_info* info,
                             void* stream);

/* ibdl_batch_solve plus the grid solutions, as ibdl_solve_grid per instance.
 * u: per instance a device [nrhs_i][n_i^dim_i] array. */
ibdl_status ibdl_batch_solve_grid(ibdl_batch batch, const double* const* data, const double* const* g,
                                  const ibdl_solve_opts* opts, double* const* sol, double* const* u,
                                  ibdl_solve_info* info, void* stream);

/* ibdl_eval_grid for every instance (FP64; async after the wait).  vb: per
 * instance, required for Neumann instances (may be NULL when none is Neumann);
 * g: NULL or per instance with NULL entries allowed. */
ibdl_status ibdl_batch_eval_grid(ibdl_batch batch, const double* const* sol, const double* const* vb,
                                 const double* const* g, double* const* u, void* stream);

/* Stage timing of the batch's grid passes, as ibdl_plan_set_timing / ibdl_plan_stage_times. */
ibdl_status ibdl_batch_set_timing(ibdl_batch batch, int32_t enable);
ibdl_status ibdl_batch_stage_times(ibdl_batch batch, double* ms_host, const char** names,
                                   int64_t* calls, int32_t cap, int32_t* count);

/* ---------------------------------------------------------------------------
 * Serving: a worker thread admits solve requests (any dimension, grid size,
 * geometry, boundary condition, precision) first come first served while the
 * sum of the admitted requests' footprints (ibdl_server_footprint) stays within
 * the memory budget and fewer than max_slots are on the device.  Requests
 * admitted at the same scheduling step form a cohort whose solve runs as one
 * batched task on one of the server's streams; cohorts on different streams
 * overlap on the device, and new requests are admitted while others run.
 * Each request gets its own plan (built on admission), device Krylov state and
 * results; these are the same as ibdl_solve + ibdl_eval_grid through a plan of
 * its own (bit-identical: a right-hand side's arithmetic does not depend on its
 * cohort).  Entry points may be called from any host thread.
 * ------------------------------------------------------------------------- */

typedef struct {
    double queue_ms;       /* submission -> admission                                  */
    double run_ms;         /* admission -> results complete on the device              */
    double total_ms;       /* submission -> results complete                           */
    int32_t cohort_size;   /* requests admitted together with this one (itself included) */
} ibdl_request_times;

typedef struct {
    int64_t submitted, completed, cohorts;
    int32_t pending, active, peak_active;
    size_t in_use_bytes, peak_in_use_bytes, budget_bytes;
} ibdl_server_stats;

/* Start a server on the current device.  hbm_budget_bytes: admission budget
 * (0: 90% of the device memory free now; more than is free: IBDL_ERR_OOM);
 * max_slots >= 1: requests on the device at once; streams in 1..16: cohorts in
 * flight at once. */
ibdl_status ibdl_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t streams, ibdl_server* out);

/* Wait for every submitted request to finish, stop the worker, free the server. */
ibdl_status ibdl_server_destroy(ibdl_server server);

/* Bytes a request is charged at admission: ibdl_plan_footprint plus its share of
 * its cohort's argument tables (host-only). */
ibdl_status ibdl_server_footprint(const ibdl_desc* desc, int32_t nrhs, int32_t restart, size_t* bytes);

/* Queue a solve (non-blocking): the right-hand side, GMRES (Sec. 5.3) with FP64
 * refinement for MIXED, and, when u is not NULL, the grid solution (Sec. 4.2, step 2).
 * desc, data [nrhs][M], g [nrhs][n^dim] or NULL, sol [nrhs][M], u [nrhs][n^dim]
 * or NULL: as for ibdl_plan_create / ibdl_solve / ibdl_eval_grid (Neumann
 * requests use data as V_b for the grid solution).  The geometry, data and g are
 * read after the work queued on `stream` so far; every buffer must stay valid
 * until the request completes.  opts->x0 must be NULL.  Errors: IBDL_ERR_ARG,
 * IBDL_ERR_OOM (footprint above the budget), IBDL_ERR_STATE (shutting down). */
ibdl_status ibdl_server_submit(ibdl_server server, const ibdl_desc* desc, int32_t nrhs, const double* data,
                               const double* g, const ibdl_solve_opts* opts, double* sol, double* u,
                               void* stream, uint64_t* ticket);

/* IBDL_ERR_STATE while the request is pending or running.  Once complete,
 * fills info (HOST [nrhs]) and times (either may be NULL), forgets the ticket
 * and returns the request's status (IBDL_OK, IBDL_ERR_NOCONV, IBDL_ERR_NUMERIC,
 * or the plan construction error).  Unknown tickets: IBDL_ERR_ARG. */
ibdl_status ibdl_server_poll(ibdl_server server, uint64_t ticket, ibdl_solve_info* info,
                             ibdl_request_times* times);

/* As ibdl_server_poll, but blocks until the request is complete. */
ibdl_status ibdl_server_wait(ibdl_server server, uint64_t ticket, ibdl_solve_info* info,
                             ibdl_request_times* times);

ibdl_status ibdl_server_get_stats(ibdl_server server, ibdl_server_stats* out_host);

/* Tile autotuner.  The row passes (spread + x-transform, x-inverse + interpolation)
 * are built in four workgroup shapes: 1, 2 and 4 right-hand sides per workgroup
 * with several lines each, and one line of one right-hand side; the first pass of
 * a new configuration (precision, dimension, n, forcing-grid input or not, output
 * kind, right-hand-side counts) runs every shape once untimed and then three
 * timed rounds over all shapes on the device, and keeps the shape with the
 * fastest run for the rest of the process.  Every shape gives bit-identical
 * results.  ibdl_set_autotune clears the choices and sets the mode: 1 tuner on,
 * 0 off (a fixed rule picks the shape), 2..5 always row shape 0..3 (for tests);
 * other values: IBDL_ERR_ARG.  ibdl_autotune_report writes the choices as text
 * lines into the HOST buffer (cap bytes, NUL-terminated) and returns the length
 * of the full report. */
ibdl_status ibdl_set_autotune(int32_t enable);
int32_t ibdl_autotune_report(char* buf, size_t cap);

/* Iteration graphs.  Once the operator pass of a solver's Krylov workspace has
 * run once (which settles the tuned variants), runs of 1, 2, 4 and 8 GMRES-Arnoldi
 * steps (Sec. 5.3: one operator application followed by the orthogonalisation of
 * the new basis vector, for every instance of the plan, batch or cohort) are
 * recorded as HIP graphs whose kernels read the base of the step index from
 * device memory; the workspace keeps them, and every later run of c steps, in
 * this and later solves, is at most one replay of each length (largest first) on
 * the solve's stream.  Results are bit-identical to launching the kernels one by
 * one.  On (1) or off (0, the default: the eager launches already keep the device
 * queue full, and replays measure no faster); solves of plans with stage timing
 * on never use graphs.  Takes effect for solves started after the call. */
ibdl_status ibdl_set_graphs(int32_t enable);
/* Process totals since load: out_host[0] = graphs recorded (four per Krylov
 * workspace and operator), out_host[1] = replays.  out_host: HOST array of 2. */
ibdl_status ibdl_graph_stats(int64_t* out_host);

/* Message for the last failing call on this host thread ("" if none). */
const char* ibdl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IBDL_H */
