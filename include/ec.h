/*
 * ec.h -- C-ABI of the MI355X (gfx950) library for the semi-explicit
 * eddy-current scheme of Dutine, Clemens and Schoeps, "Multiple right-hand
 * side techniques in semi-explicit time integration methods for transient
 * eddy current problems" (Secs. II-III).
 *
 * The magnetic vector potential is discretised on a staggered Cartesian
 * (FIT) grid with edge unknowns.  The dofs split into conducting (a_c) and
 * nonconducting (a_n) edges, giving the DAE of eq. (3).  The generalised
 * Schur complement (eq. 4) turns it into the ODE (5a), integrated by explicit
 * Euler (eqs. 6, 7).  Every step needs pseudo-inverse solves with the
 * nonconducting curl-curl matrix K_n (eq. 9), done by Jacobi-preconditioned
 * CG started from SPE (eq. 10) or POD (eqs. 11-14) vectors.
 *
 * Conventions shared by every call
 * --------------------------------
 * Status: every call returns EC_OK (0) or a negative EC_ERR_* code; the
 *   message of the last failure is ec_last_error(h).  No C++ exception
 *   crosses this boundary.
 * Edge arrays ("padded" layout): one array of 3*S elements, S =
 *   (nx+1)(ny+1)(nz+1).  Block c (0 x, 1 y, 2 z) holds the edges of direction
 *   c; inside a block the edge anchored at node (i,j,k) is at
 *   (k*(ny+1)+j)*(nx+1)+i.  Slots with i = nx (x), j = ny (y), k = nz (z)
 *   are padding.  Entries on Dirichlet (boundary-tangential) edges and padding
 *   must be zero on input and are zero on output.  The state array A holds
 *   a_c on conducting edges and a_n on nonconducting ones.
 * Memory: pointers named "dev" or documented as device pointers are HIP
 *   device memory owned by the caller, 16-byte aligned.  Host pointers are
 *   read during the call only.  The library never allocates device memory:
 *   all of its scratch lives in the caller's workspace (ec_bind).
 * Streams: after ec_bind every device call is enqueued asynchronously on the
 *   bound HIP stream, except where a call says it synchronises.  Handles are
 *   not thread-safe.
 */
#ifndef EC_H
#define EC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ec_problem *ec_handle;
typedef struct ec_batch_s *ec_batch;

enum {
    EC_OK = 0,
    EC_ERR_ARG = -1,            /* invalid argument or size */
    EC_ERR_HIP = -2,            /* HIP runtime failure */
    EC_ERR_NOT_CONVERGED = -3,  /* PCG reached maxit */
    EC_ERR_BREAKDOWN = -4,      /* p^T K_n p <= 0 with r != 0 */
    EC_ERR_CFL = -5,            /* dt above the bound 2/lambda_max of the last ec_cfl (eq. 8) */
    EC_ERR_NONFINITE = -6,      /* NaN or Inf in a solve or in the state */
    EC_ERR_STATE = -7,          /* call out of order (not bound, ...) */
    EC_ERR_SINGULAR_PROJ = -8   /* projected SPE/POD matrix not SPD: zero start used */
};

enum { EC_WF_DC = 0, EC_WF_SIN = 1, EC_WF_RAMP = 2, EC_WF_EXP = 3 };
enum { EC_SEQ_SRC = 0, EC_SEQ_CPL = 1, EC_SEQ_ADJ = 2, EC_SEQ_USER = 3, EC_NSEQ = 4 };
enum { EC_SV_ZERO = 0, EC_SV_PREV = 1, EC_SV_SPE = 2, EC_SV_POD = 3 };
enum { EC_PREC_FP64 = 0, EC_PREC_FP32_REFINED = 1 };
enum { EC_OP_KN = 0, EC_OP_KCN_T = 1, EC_OP_KC_KCN = 2 };
enum { EC_MASS_LUMPED = 0, EC_MASS_CONSISTENT = 1 };

#define EC_MAX_WINDOW 20

/* Uniform grid of n[0] x n[1] x n[2] cells on a box of side lengths len [m]. */
typedef struct { int32_t n[3]; double len[3]; } ec_grid;

/* Conducting material: sigma > 0 [S/m]; reluctivity nu(B) = k1 exp(k2 |B|^2)
 * + k3 [m/H] (the nonlinear nu of eq. 1; k1 = 0 gives the constant k3). */
typedef struct { double sigma, k1, k2, k3; } ec_material;

/* cell_mat (host, nx*ny*nz bytes, cell (i,j,k) at (k*ny+j)*nx+i): 0 marks a
 * nonconducting cell of reluctivity nu0, m >= 1 selects mats[m-1]. */
typedef struct {
    const uint8_t *cell_mat;
    const ec_material *mats;
    int32_t n_mats;
    double nu0;
} ec_materials;

/* Source j_S = X_S i_S(t) (eq. 1): edge_current is X_S as a host padded edge
 * array [A per unit i_S], nonzero on nonconducting edges only and discretely
 * divergence free.  i_S(t_m), t_m = m dt: DC amp; SIN amp sin(2 pi freq t);
 * RAMP amp min(1, m/ramp_steps); EXP amp (1 - exp(-t/tau)) (Sec. IV). */
typedef struct {
    const double *edge_current;
    int32_t waveform;
    double amp, freq, tau;
    int64_t ramp_steps;
} ec_source;

/* PCG options.  Stop when ||b - K_n x||_2 <= rtol ||b||_2 (recursive
 * residual).  FP32_REFINED: FP32 inner PCG to inner_rtol inside an FP64
 * residual-refinement loop of at most outer_max passes. */
typedef struct {
    double rtol;
    int32_t maxit;
    int32_t precision;
    double inner_rtol;
    int32_t inner_maxit;
    int32_t outer_max;
} ec_solve_opts;

/* Record written to device memory by every solve. */
typedef struct {
    int32_t iters;        /* PCG iterations (inner ones summed for FP32_REFINED) */
    int32_t outer_iters;  /* refinement passes (FP32_REFINED), else 0 */
    int32_t status;       /* EC_OK or EC_ERR_* */
    int32_t basis_cols;   /* SPE basis / POD modes used by the start vector */
    double rel_res;       /* final ||r|| / ||b|| */
    double b_norm;        /* ||b|| */
    double pod_info;      /* eq. (13) value of the POD truncation (else 1) */
    double r0_rel;        /* ||r_0|| / ||b|| of the start vector */
} ec_solve_info;

/* Step options: start-vector method and its window (SPE: last `window`
 * accepted solutions; POD: `window` snapshots, at most pod_kmax modes with
 * sigma_i >= pod_eps sigma_1). */
typedef struct {
    int32_t start_method;
    int32_t window;
    int32_t pod_kmax;
    double pod_eps;
    ec_solve_opts solve;
    /* PCG iterations a captured graph budgets per solve, for the source and
     * the coupling sequence; 0 = solve.maxit (at most 4096).  With a
     * smaller positive budget B, an FP64 solve of a single problem runs
     * B - 1 iteration kernels and then one persistent kernel that takes the
     * B-th iteration and any further ones up to solve.maxit (same iterates:
     * with at most one 256-node tile per block the results do not depend on
     * the budget).  An FP32-refined solve issues every outer pass up to
     * solve.outer_max (a pass after the FP64 check has passed does
     * nothing): the first inner PCG as above with B and inner_maxit, each
     * later one as one iteration kernel and the persistent kernel (passes
     * after the first are short corrections).  A solve short of its
     * tolerance at solve.maxit ends with EC_ERR_NOT_CONVERGED in its record
     * and in the worst-status counter.  Eager calls ignore these. */
    int32_t graph_iters[2];
    /* 1: a captured step runs as one chain of kernels.  0 (default): with an
     * SPE history and FP64 solves, the history pushes run on a forked
     * branch beside the other sequence's work (see ec_graph_capture_step);
     * a chain suits many different graphs launched in turn.  Eager calls
     * ignore it. */
    int32_t graph_serial;
} ec_step_opts;

/* Create a problem (host only): validates the descriptors, builds the edge
 * classes (Dirichlet / conducting / nonconducting), M_sigma, the reluctivity
 * tables and checks that X_S lies on nonconducting edges and has zero
 * discrete divergence (G^T X_S = 0, needed for a consistent right-hand side
 * of the singular K_n, Sec. II).  EC_ERR_ARG on any violation.  *out = NULL
 * on failure; ec_last_error(NULL) then holds the message. */
int32_t ec_create(const ec_grid *grid, const ec_materials *mat,
                  const ec_source *src, ec_handle *out);
int32_t ec_destroy(ec_handle h);

/* Sizes: padded edge-array length, conducting and nonconducting edge counts
 * and the workspace bytes needed for start-vector windows of up to
 * `window_cap` columns (1..EC_MAX_WINDOW). */
int32_t ec_sizes(ec_handle h, int32_t window_cap, int64_t *n_padded, int64_t *n_c,
                 int64_t *n_n, int64_t *workspace_bytes);

/* Bind a HIP stream and a caller-owned device workspace of at least
 * ec_sizes(...) bytes (256-byte aligned).  Uploads the tables and zeroes the
 * state (a = 0, empty histories); synchronises the stream.  The first bind on
 * a device also sets up the scratch of every HIP hardware queue (one stream
 * per queue, created, used by one kernel that touches no global memory, and
 * destroyed), so that no replay of a captured step waits for it.  Returns
 * EC_ERR_HIP if a HIP call fails. */
int32_t ec_bind(ec_handle h, void *hip_stream, void *workspace, int64_t bytes,
                int32_t window_cap);

/* y = op(x) on device padded arrays (y must not alias x):
 *   EC_OP_KN      y = K_n x            (x read on nonconducting edges)
 *   EC_OP_KCN_T   y = K_cn^T x_c       (x read on conducting edges), eq. (7)
 *   EC_OP_KC_KCN  y = K_c(x_c) x_c + K_cn x_n on conducting edges, with the
 *                 reluctivity evaluated at x (eq. 3, first block row). */
int32_t ec_apply(ec_handle h, int32_t op, const double *x, double *y);

/* Grad-div weight of the SPE projection (eq. 10; Sec. II names grad-div
 * regularisation as the alternative to the weak gauging of PCG).  The SPE
 * start vector solves the projected system with Q^T (K_n + eta D^T D) Q,
 * D = discrete divergence G^T at the free nodes (interior nodes that no
 * conducting edge ends on), eta = factor * (half the mean K_n diagonal of an
 * edge off the conductor).  K_n^+ b has zero divergence there, so the exact
 * solution is unchanged; the term stops the projection from amplifying the
 * gradient (null-space) part that PCG never removes from a start vector.
 * factor = 0 gives the projection as printed; the default is 1.  Solves in
 * EC_PREC_FP32_REFINED precision use 1e-6 of the weight: their solutions
 * carry a gradient part of FP32 size, which the full weight would trade for
 * range error.  An SPE history built with another weight starts anew at its
 * next push or solve.  EC_ERR_ARG for a negative or non-finite factor.
 * POD (eqs. 11-14) is unaffected: its truncation drops those directions. */
int32_t ec_set_gauge_penalty(ec_handle h, double factor);

/* PCG iteration kernel of the handle's FP64 and FP32 solves (eq. 9): 0 the
 * node-parallel kernel (one thread per node, 24-point stencil from global
 * memory), 1 the 2.5D kernel (a 256-node column per block marching over a
 * chunk of planes, the stencil input staged once per plane in LDS), -1 the
 * default choice (2.5D from 96^3 nodes).  Both compute the same iteration
 * (results agree to rounding of the partial sums).  EC_ERR_ARG for another
 * kind or a grid the 2.5D grid does not fit. */
int32_t ec_set_pcg_kernel(ec_handle h, int32_t kind);

/* Autotuner of the handle's FP64/FP32 PCG iteration kernel: times one
 * iteration (every iteration active, scratch vectors) for the node-parallel
 * kernel and the 2.5D kernel with columns of 16x16, 32x8 and 64x4 nodes and
 * 4, 8, 16 or 32 planes per block (grids within the block limit), and keeps
 * the fastest.  With cache_path it first looks for a pick recorded for this
 * device and grid and appends new picks (one text line each).  Outputs:
 * column width (0 = node-parallel), planes per block, microseconds per
 * iteration.  The handle's stepping state is untouched. */
int32_t ec_tune_pcg(ec_handle h, const char *cache_path, int32_t *ti, int32_t *kb, double *us);

/* Linear-independence threshold of the SPE window (eq. 10 asks for linearly
 * independent solutions without a number): a pushed solution x joins the
 * basis only if its part orthogonal to the basis exceeds tol * ||x||.
 * Default 1e-10 (FP64 round-off of consecutive solutions); solutions from
 * FP32-refined solves carry FP32-level noise and want a larger value.
 * Applies to later pushes.  EC_ERR_ARG unless 0 < tol < 1. */
int32_t ec_set_dependency_tol(ec_handle h, double tol);

/* Sequence histories (eq. 9: one history per right-hand-side sequence).
 * reset empties it; push appends a solution x (device padded array). */
int32_t ec_history_reset(ec_handle h, int32_t seq);
int32_t ec_history_push(ec_handle h, int32_t seq, int32_t method, int32_t window,
                        const double *x);

/* x0 from the history of `seq`: SPE (eq. 10) or POD (eq. 14) Galerkin
 * projection x0 = U (U^T K_n U)^{-1} U^T b; an empty history gives x0 = 0.
 * info (device, may be NULL) receives basis_cols, pod_info and r0_rel. */
int32_t ec_start_vector(ec_handle h, int32_t seq, int32_t method, int32_t window,
                        int32_t pod_kmax, double pod_eps, const double *b, double *x0,
                        ec_solve_info *dev_info);

/* K_n x = b by Jacobi-PCG (eq. 9).  method: ZERO (x0 = 0), PREV (x holds the
 * start), SPE/POD (start from the history, then push the solution).
 * dev_info (device, may be NULL) receives the record.  Asynchronous: a
 * non-converged solve is reported in the record, not in the return value. */
int32_t ec_solve(ec_handle h, int32_t seq, int32_t method, int32_t window,
                 const double *b, double *x, const ec_solve_opts *opts,
                 ec_solve_info *dev_info);

/* Replace the state: A (device padded) becomes a^{m-1}; recomputes
 * K_n^+ K_cn^T a_c (zero-start solve at opts->rtol) and empties histories.
 * Synchronises. */
int32_t ec_set_state(ec_handle h, const double *A, const ec_solve_opts *opts);

/* One explicit Euler step m (eqs. 6 and 7, with the sign of eq. 5a):
 *   s_j = K_n^+ j^m;  g = K_c(a_c) a_c + K_cn (s_j - s_c);
 *   a_c^m = a_c^{m-1} - dt M_c^{-1} g;  s_c = K_n^+ K_cn^T a_c^m;
 *   a_n^m = s_j - s_c.
 * A (device) holds a^{m-1} on entry and a^m on exit; it must be the array of
 * the previous step (or of ec_set_state).  m < 0 takes the step index from
 * the device counter (advanced by every step).  dev_info (device, may be
 * NULL) receives two records: the source and the coupling solve. */
int32_t ec_step(ec_handle h, int64_t m, double dt, double *A, const ec_step_opts *opts,
                ec_solve_info *dev_info);

/* nsteps steps m0+1..m0+nsteps without host synchronisation; dev_info, if
 * not NULL, receives 2*nsteps records. */
int32_t ec_run(ec_handle h, int64_t m0, int64_t nsteps, double dt, double *A,
               const ec_step_opts *opts, ec_solve_info *dev_info);

/* Set the device step counter to m (the last completed step): the next
 * step with a negative m, or the next replay of a captured step, is m+1. */
int32_t ec_set_step(ec_handle h, int64_t m);

/* Device-side totals since bind or the last reset: solves, PCG iterations
 * per sequence, worst status.  Synchronises. */
int32_t ec_counters(ec_handle h, int64_t *n_steps, int64_t *iters_src, int64_t *iters_cpl,
                    int64_t *iters_adj, int32_t *worst_status);
int32_t ec_counters_reset(ec_handle h);

/* Largest eigenvalue of M_c^{-1} K_S(a_c) (eq. 8) by the power method with
 * `power_iters` iterations (each one K_n^+ solve), reluctivity frozen at A.
 * Synchronises; result in *lambda_max (host).  The handle keeps the value:
 * from then on every step (ec_step, ec_run, captures, batch steps, the
 * adjoint's forward pass) with dt * lambda_max > 2, outside the explicit
 * Euler bound of eq. 8, fails with EC_ERR_CFL before any work is enqueued.
 * ec_bind and ec_set_material clear it (no check until the next ec_cfl). */
int32_t ec_cfl(ec_handle h, const double *A, int32_t power_iters, double rtol,
               double *lambda_max);

/* Implicit Euler step m with Newton's method: the reference the paper
 * compares the semi-explicit scheme with (Secs. I and IV).  With a_n
 * eliminated as in eqs. (4)-(5b), the conducting unknowns a^m solve
 *   F(a) = M_c (a - a^{m-1})/dt + N(a) - S a + K_cn K_n^+ j^m = 0
 * (N(a) = [C^T M_nu(a) C a]_C, S = K_cn K_n^+ K_cn^T); Newton takes
 * J d = -F, J = M_c/dt + J_N(a) - S, from a = a^{m-1} until
 * ||F|| <= newton_rtol ||F(a^{m-1})|| or max_newton iterations, each system
 * by GMRES(gmres_m) (left-preconditioned by (M_c/dt)^-1, restarted, at most
 * gmres_max Arnoldi steps per Newton iteration) to gmres_rtol of its
 * preconditioned right-hand side; every product with J solves K_n^+ once
 * (from zero, inner_rtol), every Newton iteration once more for s_c(a) (on
 * the coupling sequence, started as start_method / window say, like the
 * source solve s_j = K_n^+ j^m on the source sequence); then
 * a_n^m = s_j - s_c(a^m).  A (device padded) holds a^{m-1} on entry and a^m
 * on exit; the step counter advances as for ec_step.  Unconditionally
 * stable: dt is free of the bound of eq. (8).  *info (host, may be NULL)
 * receives the counts and the first and last ||F|| (status
 * EC_ERR_NOT_CONVERGED if max_newton was reached first).  Uses the lumped
 * M_c and a fixed dt (EC_ERR_STATE otherwise); not capturable.
 * Synchronises (the Newton and GMRES stopping tests read device norms).
 * With SPE- or POD-started coupling solves the error of s_c(a) lies outside
 * the window rather than spread like a zero-started solve's, and ||F||
 * levels off near inner_rtol times the conditioning: keep newton_rtol above
 * about 100 inner_rtol there. */
typedef struct {
    double newton_rtol;
    int32_t max_newton;
    int32_t gmres_m;        /* restart length, 1..20 */
    int32_t gmres_max;      /* Arnoldi steps per Newton iteration */
    double gmres_rtol;
    double inner_rtol;      /* K_n^+ solves */
    int32_t start_method;   /* EC_SV_*: source and coupling solves */
    int32_t window;
} ec_implicit_opts;
typedef struct {
    int32_t newton_iters, gmres_iters, kn_solves, status;
    double res0, res;
} ec_implicit_info;
int32_t ec_implicit_step(ec_handle h, int64_t m, double dt, double *A, const ec_implicit_opts *o,
                         ec_implicit_info *info);

/* Device-side estimate of the explicit Euler bound (eq. 8; the paper finds
 * lambda_max by the power method) at state A (device padded; its conducting
 * part sets the reluctivity): `iters` power iterations on
 *   jacobian = 1: M_c^{-1} (J_N(A) - S), J_N the derivative of
 *                 N(a) = [C^T M_nu(a) C a]_C (the step linearised at A);
 *   jacobian = 0: M_c^{-1} (K_c(nu(A)) - S) = M_c^{-1} K_S(A) of eq. (8),
 * S = K_cn K_n^+ K_cn^T, run as the transpose (X^T - S) M_c^{-1} (same
 * eigenvalues) with Euclidean normalisation on the device: no host copies
 * or synchronisation beyond those of eager PCG solves.  Each iteration is
 * one K_n^+ solve (rtol) of the EC_SEQ_USER sequence, whose history the call
 * resets, started as `method` says (EC_SV_ZERO, EC_SV_PREV or EC_SV_SPE over
 * `window` columns: consecutive right-hand sides converge, so SPE starts
 * shorten the solves).  *lambda_dev (device double) receives ||B v|| for the
 * unit iterate v after each iteration (|lambda|_max in the limit);
 * rec_dev (device, 2 * iters doubles, may be NULL) the pairs
 * (||B v||, v^T B v) per iteration.  Asynchronous; not capturable
 * (EC_ERR_STATE under capture).  EC_ERR_ARG for bad arguments or a problem
 * without conducting edges. */
int32_t ec_cfl_estimate(ec_handle h, const double *A, int32_t iters, double rtol, int32_t method,
                        int32_t window, int32_t jacobian, double *lambda_dev, double *rec_dev);

/* Adaptive steps: with lambda_dev (device double, e.g. the output of
 * ec_cfl_estimate, re-estimated whenever the caller likes) every later step
 * of the handle (eager, captured or batched) reads it on the device and
 * takes dt_m = dt 2^-k with the smallest k >= 0 such that
 * dt_m * lambda <= 2 * safety, dt being the step call's argument (the
 * largest step); a non-positive or non-finite lambda leaves dt_m = dt.  The
 * source time advances as t_m = t_{m-1} + dt_m (ramp sources stay indexed by
 * m), and the EC_ERR_CFL check of ec_cfl does not apply.  lambda_dev = NULL
 * returns to fixed steps (t_m = m dt).  0 < safety <= 1 (EC_ERR_ARG
 * otherwise).  The handle keeps the pointer: it must stay valid while steps
 * run.  The adjoint calls do not support adaptive steps. */
int32_t ec_set_adaptive_dt(ec_handle h, const double *lambda_dev, double safety);

/* Step index m, source time t_m and step dt_m of the last step (host
 * outputs, each may be NULL).  t restarts at 0 with ec_set_state.
 * Synchronises. */
int32_t ec_clock(ec_handle h, int64_t *m, double *t, double *dt);

/* Conductivity matrix M_c of the step (eq. 6).  EC_MASS_LUMPED (default):
 * the diagonal FIT matrix, M_c^{-1} an edge-wise scale.  EC_MASS_CONSISTENT:
 * the mass matrix of the lowest-order edge elements on the conducting cells
 * (per cell and direction sigma h_a1 h_a2 / h_c times 1/9, 1/18 or 1/36 for
 * an edge with itself, a side apart or diagonally across the transverse
 * face; its row sums are the lumped matrix), non-diagonal: every step then
 * solves M_c y = g for its update (the last paragraph of Sec. III names
 * M_c^{-1} as a further right-hand-side sequence), by Jacobi-PCG (same
 * single-reduction form as the K_n solves) to rtol, at most maxit
 * iterations (a captured step issues maxit iteration kernels), started
 * from zero (EC_SV_ZERO) or from the SPE projection with M_c over the last
 * `window` solutions of that sequence (EC_SV_SPE, eq. 10 with M_c in place
 * of K_n).  Resets that history.  Batch steps, the adjoint and the CFL
 * estimates (ec_cfl, ec_cfl_estimate) use the lumped matrix (batches and the
 * adjoint refuse a consistent one with EC_ERR_STATE).  EC_ERR_ARG for bad
 * values.
 * ec_mass_apply: y = M_c x on the conducting edges (device padded arrays;
 * y's other entries are left as they are).
 * ec_mass_solve: M_c y = g (device padded, conducting entries) with the
 * configured start and tolerance, pushing y into the sequence's history;
 * dev_info (device, may be NULL) receives the record.
 * ec_mass_counters: solves with the consistent M_c and their PCG
 * iterations since bind or ec_counters_reset (synchronises). */
int32_t ec_set_mass(ec_handle h, int32_t kind, int32_t method, int32_t window, double rtol,
                    int32_t maxit);
int32_t ec_mass_apply(ec_handle h, const double *x, double *y);
int32_t ec_mass_solve(ec_handle h, const double *g, double *y, ec_solve_info *dev_info);
int32_t ec_mass_counters(ec_handle h, int64_t *solves, int64_t *iters);

/* Replace material mat_id (1..n_mats) of the handle: conductivity and
 * Brauer coefficients (eq. 1).  M_sigma of the conducting edges is rebuilt;
 * the conducting edge set, K_n and the start-vector histories stay valid
 * (sigma must stay positive).  A dt from ec_cfl may no longer be stable.
 * Synchronises.  EC_ERR_ARG for a bad id or values. */
int32_t ec_set_material(ec_handle h, int32_t mat_id, const ec_material *m);

/* Discrete adjoint of the time loop (eqs. 6-7, sign of eq. 5a) for the
 * Joule loss of the conductor
 *     L = sum_{m=1..n_steps} (1/dt) d_m^T M_c d_m,   d_m = a_c^m - a_c^{m-1},
 * and its gradient with respect to the conductivity sigma and the Brauer
 * coefficient k1 of one material.  With mu_m = dL/da_c^m:
 *     mu_M = (2/dt) M_c d_M,
 *     mu_m = (2/dt) M_c (d_m - d_{m+1}) + mu_{m+1} - dt [J_N(a^m)^T - S] M_c^{-1} mu_{m+1},
 * N(a) = [C^T M_nu(a) C a]_C, S = K_cn K_n^+ K_cn^T (one K_n^+ solve per
 * step on sequence EC_SEQ_ADJ with the step options' start vector), and
 *     dL/dsigma = sum_m [(1/dt) d_m^T Phi d_m - mu_m^T M_c^{-1} Phi d_m],
 *     dL/dk1    = -dt sum_m mu_m^T M_c^{-1} dN/dk1(a^{m-1}),   Phi = dM_c/dsigma.
 *
 * ec_adjoint_sizes: bytes of the caller-owned device workspace for n_steps
 * steps with a checkpoint every checkpoint_every steps (one per segment:
 * a_c, s_c, s_j and the source / coupling histories, so that a recomputed
 * segment is bitwise the forward one).
 * ec_adjoint_forward: a^0 from A (conducting part; like ec_set_state), then
 * steps 1..n_steps (ec_step semantics, eager), writing the checkpoints and
 * *loss (device double).  A holds a^M on return.
 * ec_adjoint_backward: with the same workspace, n_steps, checkpoint_every and
 * dt as the last forward call (EC_ERR_STATE otherwise), recomputes each
 * segment from its checkpoint (last first) and runs the adjoint recursion;
 * grads (device double[2]) = {dL/dsigma, dL/dk1} of material mat_id.  It
 * leaves the stepping state of a recomputed segment behind: call
 * ec_set_state before stepping again.  EC_ERR_ARG for bad sizes, ids or a
 * workspace below ec_adjoint_sizes; EC_ERR_NONFINITE when the loss or the
 * gradients are not finite (a diverging run).  Both synchronise. */
int32_t ec_adjoint_sizes(ec_handle h, int64_t n_steps, int32_t checkpoint_every, int64_t *bytes);
int32_t ec_adjoint_forward(ec_handle h, int64_t n_steps, double dt, int32_t checkpoint_every,
                           const ec_step_opts *opts, void *adj_ws, int64_t adj_bytes, double *A,
                           double *loss);
int32_t ec_adjoint_backward(ec_handle h, int64_t n_steps, double dt, int32_t checkpoint_every,
                            const ec_step_opts *opts, void *adj_ws, int64_t adj_bytes,
                            int32_t mat_id, double *grads);

/* Batches of independent problems (uneven grids, materials and dt, e.g. the
 * samples of a multi-query study) stepped together on one stream: every
 * PCG iteration of all instances' source (or coupling) solves is one
 * launch, each instance on its own slice of the grid with the arithmetic of
 * a single-instance solve (a batched instance equals the same problem
 * stepped alone, bitwise); start vectors, the conducting update and the
 * histories run as each instance's kernels.  FP64 solves only.
 *
 * ec_batch_sizes / ec_batch_create: n bound handles (all bound to the same
 * stream) and a caller-owned device workspace of ec_batch_sizes bytes
 * (256-byte aligned).  The batch borrows the handles (destroy it first) and
 * sets the PCG iteration grid of each (its tiles per block, see
 * ec_batch_set_tiles); ec_set_pcg_kernel(h, -1) gives a handle back its
 * default grid for stepping alone.
 * ec_batch_step / ec_batch_run: dt[i] (host array) and A[i] (host array of
 * device state pointers) per instance; m < 0 (step) or m0 < 0 (run) takes
 * each instance's step index from its device counter.  Per-instance
 * counters (ec_counters) record the solves.  Eager calls synchronise once
 * per handful of iterations to stop when every solve has finished.
 * ec_batch_graph_capture: one step of every instance as one HIP graph
 * (device step counters; opts->graph_iters = batched iteration launches per
 * solve, 0 = solve.maxit up to 4096).  With a budget B below solve.maxit the
 * graph issues B - 1 batched iteration launches and then one persistent
 * launch that runs the B-th and every further iteration of each unfinished
 * instance over the same block map and iteration bodies (a grid barrier
 * between iterations) until all have finished or reached solve.maxit: the
 * results are those of eager batch steps, bitwise, whatever the budget, and
 * a budget of 1 makes each batched PCG solve one persistent launch after
 * its init.  Launch with ec_graph_launch.
 * ec_batch_set_tiles / ec_batch_autotune: the tiles of 256 nodes each block
 * of a batched iteration sweeps (1..64).  The autotuner times 1, 2, 4 and 8
 * on the batch itself, each as one iteration launch with every solve active
 * and one with every solve finished, and keeps the one with the least
 * active + 8 x finished time (a captured batch step issues several launches
 * in which most solves have finished for each one in which all work);
 * *us_per_iter is the active time of the pick.  With cache_path it first looks
 * for a pick recorded for this device and batch shape and appends new picks
 * (one text line each), so a cached batch always gets the same config.
 * Errors: EC_ERR_ARG / EC_ERR_STATE; the message is ec_last_error(NULL). */
int32_t ec_batch_sizes(int32_t n, const ec_handle *handles, int64_t *bytes);
int32_t ec_batch_create(int32_t n, const ec_handle *handles, void *workspace, int64_t bytes,
                        ec_batch *out);
int32_t ec_batch_destroy(ec_batch b);
int32_t ec_batch_step(ec_batch b, int64_t m, const double *dt, double *const *A,
                      const ec_step_opts *opts);
int32_t ec_batch_run(ec_batch b, int64_t m0, int64_t nsteps, const double *dt, double *const *A,
                     const ec_step_opts *opts);
int32_t ec_batch_graph_capture(ec_batch b, const double *dt, double *const *A,
                               const ec_step_opts *opts, void **graph_exec);
int32_t ec_batch_set_tiles(ec_batch b, int32_t tiles_per_block);
int32_t ec_batch_autotune(ec_batch b, const char *cache_path, int32_t *tiles_per_block,
                          double *us_per_iter);

/* HIP graph of one step (device step counter, fixed dt and opts) captured on
 * the bound stream; launch replays it on `hip_stream` (the bound stream).
 * With an SPE history, FP64 solves and opts->graph_serial = 0 the graph
 * forks (POD steps, measured slower forked, are captured as one chain; so
 * are FP32-refined solves): the history pushes run on a
 * side stream of the library beside the other sequence's work (the previous
 * step's coupling push beside the source start and solve, the source push
 * beside the coupling start and solve), so a launch leaves its own coupling
 * solution due for a push; the next launch makes it first, and every other
 * call on the handle that reads or changes the histories, the solutions or
 * what a push computes (solve, start vector, history calls, step, run,
 * set_state, set_material, set_gauge_penalty, set_dependency_tol, tuning,
 * adjoint and batch calls) makes it before its own work.  The results are
 * those of eager steps.  A graph refers to the problem's buffers and state:
 * destroy it before the problem; graph_exec is an opaque handle. */
int32_t ec_graph_capture_step(ec_handle h, double dt, double *A, const ec_step_opts *opts,
                              ec_solve_info *dev_info, void **graph_exec);
int32_t ec_graph_launch(void *graph_exec, void *hip_stream);
int32_t ec_graph_destroy(void *graph_exec);

/* Allocation-free PCG solve, for callers that cannot allocate device
 * memory or take a workspace of their own: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  It is ec_solve's
 * FP64 Jacobi-PCG of K_n x = b (eq. 9) with method EC_SV_ZERO (x0 = 0) or
 * EC_SV_PREV (x holds the start), same kernels and results, but its seven
 * iteration vectors, control records and block partials live in a static
 * device array of EC_STATIC_SCRATCH_BYTES in the library (one per GPU,
 * held until the process ends) instead of the handle's workspace.  The
 * grid is limited by that array: n_padded at most EC_STATIC_MAX_NPAD
 * (e.g. 72^3 cells); a larger handle gets EC_ERR_ARG, as do other methods,
 * FP32_REFINED precision or unaligned pointers.  b, x (device, padded) and
 * dev_info (device, may be NULL) are the caller's; the handle must be bound
 * (its tables and stream are used; its counters are not updated).  No
 * hipMalloc, hipFree or allocating call is made.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (several streams,
 * threads or handles) race; calls in stream order do not.  Asynchronous
 * like ec_solve (eager calls poll the device done flag; under capture the
 * solve budget and the persistent tail apply as in a captured step). */
#define EC_STATIC_SCRATCH_BYTES (64ll << 20)
#define EC_STATIC_MAX_NPAD 1195904
int32_t ec_solve_static(ec_handle h, int32_t method, const double *b, double *x,
                        const ec_solve_opts *opts, ec_solve_info *dev_info);

/* Message of the last failure on h (or of the last ec_create if h = NULL). */
const char *ec_last_error(ec_handle h);

#ifdef __cplusplus
}
#endif
#endif
