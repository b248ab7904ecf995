// ec_internal.h -- device-side data structures and kernel launchers of the
// gfx950 library (private to the library; the public boundary is ec.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ec.h"

namespace ec {

constexpr int kMaxWin = EC_MAX_WINDOW + 4;   // columns of the small matrices
                                             // (window + the column being added)
constexpr int kMaxMat = 16;              // materials incl. id 0
constexpr int kTile = 256;               // nodes per tile = threads per block
constexpr int kMdBlocks = 256;           // grid of the basis-product kernels
constexpr int kMdStride = 2 * kMaxWin;  // partial values per block
constexpr int kMaxBlocks = 2048;        // grid cap of node kernels (multiple of 8)
constexpr int kHaloMax = 256;           // one-tile iterations stage a halo of px <= this in LDS

// Grid geometry and the constant-coefficient stencil of the nonconducting
// region.  Every face touching a nonconducting edge lies between two
// nonconducting cells, so K_n and K_cn^T use the single reluctivity nu0.
struct Geo {
    int nx, ny, nz;
    int px, py;              // nx+1, ny+1 (node strides)
    int64_t S;               // entries per direction block = node count
    int64_t npad;            // 3*S
    double hx, hy, hz;
    double wx, wy, wz;       // nu0 * (dual length / area) of x/y/z-normal faces
    double dinv[3];          // Jacobi: 1/diag(K_n) of x/y/z edges
    int box;                 // conductor is an axis-aligned box of cells
    int clo[3], chi[3];      // that box (cells, inclusive); clo > chi: none
    const uint8_t *cls;      // edge classes when box == 0
};

// Materials: per id reluctivity coefficients and conductivity.
struct Mats {
    double sig[kMaxMat], k1[kMaxMat], k2[kMaxMat], k3[kMaxMat];
    double nu0;
    int n;
};

// Device-resident state of one right-hand-side sequence.
//  SPE: Q columns (raw, orthogonal) with scales s_i (q_i = s_i Q_i), KQ the
//       K_n products of the raw columns; H = q^T K q (normalised); R the
//       window coordinates (X_window = q R, upper triangular k x k).
//  POD: ring of raw snapshots X and K X; G = X^T X, H = X^T K X.
struct SeqDev {
    int method, cap, k, w;
    int accept, rotate, active, flags;
    int kpod, head, count, status;
    int ncol_md;             // columns handed to the next basis product
    int npush;               // POD: ring columns of the next push (incl. the new slot)
    int zero_start;          // 1: the start vector is zero
    int pad1;
    double xnorm, rho, pod_info, r0_rel;
    double pod_eps;
    // largest diagonal entry of K_n: the projected matrices are U^T K_n U (plus
    // the grad-div term) for unit-norm columns, so a Cholesky pivot at or below
    // 1e-14 of max(hscale, largest diagonal of the matrix) marks it singular
    // (a window of null vectors alone has a tiny diagonal of its own)
    double hscale;
    int pod_kmax, pad2;
    double s[kMaxWin + 1];
    double H[kMaxWin * kMaxWin];
    double R[kMaxWin * kMaxWin];
    double G[kMaxWin * kMaxWin];
    double V[kMaxWin * kMaxWin];
    double lam[kMaxWin];
    double c1[kMaxWin + 1], c2[kMaxWin + 1];
    double cA[kMaxWin + 1], cB[kMaxWin + 1];   // lincomb coefficients
    double a1, a2;                              // lincomb scalars
    double rot[kMaxWin * kMaxWin];              // basis rotation (SPE downdate)
    int rot_in, rot_k;                          // columns in / kept by the rotation
    int slot_new;                               // column slot being filled
    // 1 while the solution of the sequence's last start is due for a push:
    // set by the start, cleared by the last kernel of the push (so a push
    // that was already made is skipped when it is issued again, as by a
    // graph replay that pushes the previous step's solution), and for SPE
    // also by an FP64 solve that needed no PCG iteration (its solution is the
    // start vector, which lies in span(q), so the dependency test of the
    // push would reject it); the push kernels are gated on it
    int push_on;
    // SPE: Cholesky factor of H (lower, leading dimension kMaxWin) made by
    // the last kernel of a push; valid while L_ver == H_ver (H_ver counts
    // the pushes that changed H); chol_bad: H not numerically definite
    int H_ver, L_ver, chol_bad, pad3;
    double L[kMaxWin * kMaxWin];
};

// Per-handle control block in device memory.
struct Ctrl {
    int64_t step;            // step counter m
    double scale;            // i_S(t_m) of the current step
    double one;              // constant 1.0 (scale of unscaled right-hand sides)
    double dt;
    int64_t n_steps;
    int64_t iters[EC_NSEQ];
    int worst;               // most severe status seen (most negative)
    int pad;
    int refine_done;         // FP32-refined outer loop finished flag
    int refine_zero;         // the right-hand side was zero
    double refine_rr, refine_bb;
    double refine_tol;       // relative tolerance of the next inner FP32 solve
    double t;                // time t_m of the current step (adaptive steps accumulate it)
    int64_t mass_solves, mass_iters;   // solves with the consistent M_c and their iterations
};

// ----------------------------------------------------------------- launchers
struct Vec2 {
    const double *p;
    const double *scale;     // device scalar or nullptr (=1)
};

void spmv(const Geo &g, const double *x, double *y, const int lo[3], const int hi[3],
          hipStream_t st);
// y (if given) = K_n x over the full grid; ycopy/xcopy (if given) receive
// K_n x and x at column *slot (ld apart); ypen (if given) = K_n x + eta D^T D x
// on nonconducting edges (D: divergence at free nodes; K_n x for eta = 0).
// Nothing happens for a set whose *active == 0.  s1: a second, independent
// set in the same launch.
struct SlotArgs {
    const double *x;
    double *y, *ycopy, *xcopy, *ypen;
    const int *slot, *active;
    double eta;
    // if pre_seq: every block first runs the acceptance test of an SPE push
    // (OP_SPE_PUSH3, |x|^2 from the partials pin, dependency tolerance tol)
    // and leaves unless the column is accepted (active unused); block 0
    // stores the test's results
    SeqDev *pre_seq;
    const double *pin;
    double tol;
};
void spmv_slots(const Geo &g, int64_t ld, const SlotArgs &s, hipStream_t st,
                const SlotArgs *s1 = nullptr);
// one set per instance of a batch, each on its own grid (full box)
struct SlotTab {
    Geo g;
    int64_t ld;
    SlotArgs s;
};
// grid covers the largest instance; tpx_max = max over the table of
// ceil(tiles / 8) with tiles = ceil((nx+1)(ny+1)(nz+1) / 256)
void spmv_slots_tab(const SlotTab *tab, int n, int tpx_max, hipStream_t st);
int spmv_slot_tpx(const Geo &g);
// y = K_n x over the box [lo, lo + ext) of each instance of a batch (ext of 0
// cells: no work); grid from the largest box
struct BoxTab {
    Geo g;
    int lo[3], ext[3];
    const double *x;
    double *y;
};
int spmv_box_tpx(const int ext[3]);
void spmv_box_tab(const BoxTab *tab, int n, int tpx_max, hipStream_t st);
void spmv_f(const Geo &g, const float *x, float *y, hipStream_t st);

// PCG start modes
enum { START_ZERO = 0, START_X = 1, START_R = 2, START_DEV = 3, START_R2 = 4 };

// Device control record of one CG solve, double buffered by kernel parity:
// kernel i reads ctl[i & 1] and writes ctl[(i + 1) & 1].
struct CgCtl {
    double alpha, gamma, rho, bb, tol2, rho0, pad0, pad1;
    int it, done, status, zero_x;
    int pad2[4];
};

// Jacobi-PCG in the single-reduction form (Chronopoulos-Gear): one kernel
// per iteration; r, w = K_n D^-1 r and s = K_n p double buffered.  Every
// kernel reduces the block partials of the previous one (no atomics).
template <typename T>
struct CgArgs {
    Geo g;
    T *x, *p;
    T *rb[2], *wb[2], *sb[2];
    const T *b;
    const double *bscale;    // device scalar multiplying b (nullptr: 1)
    int mode;                // START_*
    SeqDev *seq;       // START_DEV reads seq->zero_start; basis info
    double rtol;
    const double *rtol_dev;  // device tolerance read at the first iteration (nullptr: rtol)
    int maxit;
    CgCtl *ctl;              // [2]
    double *part;            // [2][blocks][4]
    ec_solve_info *info;     // may be nullptr
    Ctrl *ctrl;              // accumulators (may be nullptr)
    int seq_id;
    int accum;               // add iterations to info->iters (inner refinement solves)
    const int *skip;         // device flag: nonzero -> kernels return at once
    // partials of the start combination that wrote x0 and r0 (value-major
    // rows |x0|^2, |r0|^2, |b|^2 over kMdBlocks blocks), or nullptr: the init
    // kernel stops a solve whose start already meets the tolerance
    const double *start_part;
    int tiles;
    int blocks;
    unsigned *bar;           // grid-barrier words of the tail kernel (kBarWords x kBarStride)
    // 2.5D iteration kernel (large grids): TI of the node column (0: the
    // node-parallel kernel), planes per block and the tile counts; the 2.5D
    // grid is `blocks`
    int t25, kb25, nti25, ntj25, ntk25;
};

// grid barrier of the persistent tail kernel: per-XCD population, arrival
// and release words for up to kBarXcc XCDs, one counter and one release
// word for the whole grid, each kBarStride words apart (separate 128-byte
// lines); bounded waits
constexpr int kBarStride = 32;
constexpr int kBarXcc = 16;
constexpr int kBarWords = 3 * kBarXcc + 2;
constexpr long kSpinLimit = 1L << 22;

template <typename T>
void cg_init(const CgArgs<T> &a, hipStream_t st);
template <typename T>
void cg_iter(const CgArgs<T> &a, int i, hipStream_t st);
template <typename T>
void cg_fin(const CgArgs<T> &a, int iters, hipStream_t st);
// batched iteration: all solves of a batch, one launch (block map inst/off)
void cg_iter_batch(const CgArgs<double> *tab, const int *inst, const int *off, int total_blocks,
                   int it, bool one_tile, hipStream_t st);
// *flag (device int) = 1 if every solve of tab[0..n) finished before iteration it
// init (in `mode`) / final record of every solve of a batch in one launch
void cg_init_batch(const CgArgs<double> *tab, const int *inst, const int *off, int total_blocks,
                   int mode, hipStream_t st);
void cg_fin_batch(const CgArgs<double> *tab, int n, int iters, hipStream_t st);
void batch_done(const CgArgs<double> *tab, int n, int it, int *flag, hipStream_t st);
// iterations it0.. of every unfinished solve of a batch in one persistent
// launch over the block map (grid: at most cg_tail_batch_blocks(), all
// resident; the barrier words are tab[0].bar); 0 blocks: not available
int cg_tail_batch_blocks();
hipError_t cg_tail_batch(const CgArgs<double> *tab, int n, const int *inst, const int *off,
                         int total, int it0, int blocks, bool one_tile, hipStream_t st);
// blocks of the persistent tail (at most two per CU, all resident at once, a
// multiple of 8; 0 on failure)
template <typename T>
int cg_tail_blocks();
// iterations it0.. of an unfinished solve in one persistent launch
template <typename T>
hipError_t cg_tail(const CgArgs<T> &a, int it0, int blocks, hipStream_t st, bool fin);

// basis products  C = [A_0..A_{p-1}, a_extra]^T [B_0..B_{nb-1}]  (FP64 MFMA)
struct MdArgs {
    const double *A;
    int64_t ld;
    const int *kp;           // column count on device (nullptr: kfix)
    int kfix;
    const double *a_extra;
    Vec2 B[4];
    int nb;
    const int *active;       // device flag (nullptr: always)
    double *part;
    int64_t n;
};
// a1: a second, independent argument set run in the same launch; the _tab
// launchers run the n sets of a device table (block row y = set y)
void multidot(const MdArgs &a, hipStream_t st, const MdArgs *a1 = nullptr);
void multidot_tab(const MdArgs *tab, int n, hipStream_t st);

// y1 = a1 v1 + sum cA_i A_i ; y2 = a2 s2 v2 - ... (see kernel) with partial norms
struct LcArgs {
    const double *A, *B;
    int64_t ld;
    const int *kp;
    const double *cA, *cB;
    const double *a1, *a2;   // device scalars
    const double *v1;
    Vec2 v2;
    double *y1, *y2;
    const int *active;
    const int *slot;         // if not null, y1 is column *slot of A
    int want_dots;           // partial dots A_i^T y1 (i < k) and |y1|^2
    double *part;
    int64_t n;
    // if pre_seq: every block first runs the dense step pre_op (OP_SPE_PUSH1
    // or OP_SPE_PUSH2) of that SPE sequence on the partials pin of the
    // preceding product and takes k, the coefficients, a1 and the gate from
    // it (kp, cA, a1, active unused); block 0 stores the step's results
    SeqDev *pre_seq;
    int pre_op;
    const double *pin;
};
void lincomb(const LcArgs &a, hipStream_t st, const LcArgs *a1 = nullptr);
void lincomb_tab(const LcArgs *tab, int n, bool dots, hipStream_t st);

// in-place basis rotation: columns j < k' of A (and B) become sum_i rot[i,j] A_i
struct RotArgs {
    double *A, *B;
    SeqDev *seq;
    int64_t ld, n;
};
void rotate(const RotArgs &r, hipStream_t st, const RotArgs *r1 = nullptr);
void rotate_tab(const RotArgs *tab, int n, hipStream_t st);

// dense steps on one sequence: one block reduces the partial rows of the
// preceding basis product and runs the step (for a single problem, PUSH1
// and PUSH2 run in every block of the combination that applies them, see
// LcArgs::pre_op, and PUSH3 in the slot SpMV, see SlotArgs::pre_seq)
enum {
    OP_NONE = -1,
    OP_SPE_START = 0,   // vals: Q_i^T b (k)
    OP_SPE_PUSH1,       // vals: Q_i^T x (k), x^T x
    OP_SPE_PUSH2,       // vals: Q_i^T w (k), |w|^2
    OP_SPE_PUSH3,       // vals: |x2|^2 (acceptance test)
    OP_SPE_PUSH4,       // vals: (KQ_i)^T x2, i <= k
    OP_POD_PUSH,        // vals: X_i^T x_new, X_i^T K x_new  (pairs)
    OP_POD_START,       // vals: X_i^T b (count)
    OP_RESET
};
struct SmallArgs {
    SeqDev *seq;
    int op;
    const double *part;      // partial rows of the producing product (value-major)
    int nvals;
    double tol;              // dependency threshold (SPE push)
    ec_solve_info *info;
};
void small(const SmallArgs &a, hipStream_t st, const SmallArgs *a1 = nullptr);
void small_tab(const SmallArgs *tab, int n, int op, hipStream_t st);
void seq_reset(SeqDev *seq, hipStream_t st);

// nonlinear a_c update (eq. 6) / K_c + K_cn apply over conducting edges
struct UpdArgs {
    Geo g;
    const Mats *m;           // device copy of the material table
    const uint8_t *cmat;
    const int *cslot;
    const double *minv;      // 1/M_sigma per conducting edge
    int nc;
    const double *A;         // state: a_c read on C
    const double *sj, *sc;   // y = sj - sc on N (sc may be nullptr)
    const double *xn;        // alternative N operand (apply mode), may be nullptr
    double *gout;            // if set: g on C into this compact vector, no state update
    const double *nustate;   // state whose a_c sets nu (nullptr: the operand itself)
    double *out;             // update: a_c^m on C; apply: g on C
    double dt;
    int apply;
    const Ctrl *ctrl;
};
void update_c(const UpdArgs &a, hipStream_t st);
// one launch for the n instances of a batch (nc_max: largest n_c)
void update_c_tab(const UpdArgs *tab, int n, int nc_max, hipStream_t st);

void finish_state(const Geo &g, double *A, const double *ac, const double *sj,
                  const double *sc, Ctrl *ctrl, int bump, hipStream_t st);
// lam (device scalar, may be null): adaptive step dt 2^-k, the smallest
// k >= 0 with dt_m lam <= 2 safety, and t_m = t_{m-1} + dt_m; otherwise
// t_m = m dt
void step_begin(Ctrl *ctrl, int64_t m, int wf, double amp, double freq, double tau,
                int64_t ramp, double dt, hipStream_t st, const double *lam = nullptr,
                double safety = 0.5);
// the same for the n instances of a batch, one launch each
struct FinArgs {
    int64_t n;
    double *A;
    const double *ac, *sj, *sc;
    Ctrl *ctrl;
};
void finish_state_tab(const FinArgs *tab, int n, int64_t npad_max, hipStream_t st);
struct StepArgs {
    Ctrl *ctrl;
    int wf;
    double amp, freq, tau;
    int64_t ramp;
    double dt;
    const double *lam;       // adaptive step (see step_begin), may be null
    double safety;
};
void step_begin_tab(const StepArgs *tab, int n, int64_t m, hipStream_t st);
void fill(double *y, double v, int64_t n, hipStream_t st);
// a kernel with a larger private segment than any other, touching no
// global memory (sets up a hardware queue's scratch)
void scratch_warm(hipStream_t st);
void copy_c(const int *cslot, int nc, const double *src, double *dst, hipStream_t st);
void mask_copy(const Geo &g, const double *x, double *y, int cls_keep, hipStream_t st);
// FP32-refined solve: r = b - K_n x in FP64 (and r32 = r) with block
// partials; refine_decide (one block) reduces them and sets ctrl->refine_done
void refine_residual(const Geo &g, const double *b, const double *bscale, const double *x,
                     float *r32, double *part, const Ctrl *ctrl, int blocks, hipStream_t st);
void refine_decide(const double *part, int blocks, Ctrl *ctrl, int pass, int outer_max,
                   double rtol, double inner_rtol, ec_solve_info *info, const SeqDev *seq,
                   hipStream_t st);
void refine_update(double *x, const float *d, const Ctrl *ctrl, int64_t n, hipStream_t st);
void refine_final(double *x, const Ctrl *ctrl, int64_t n, hipStream_t st);
void refine_reset(Ctrl *ctrl, hipStream_t st);
// hscale: the largest diagonal entry of K_n (scale of the projected
// matrices, whose basis columns have unit norm)
void seq_config(SeqDev *seq, int method, int cap, int kmax, double eps, double hscale,
                hipStream_t st);
// an explicit history push (not after a solve): the next push is not skipped
void seq_push_on(SeqDev *seq, hipStream_t st);
void negate(const double *x, double *y, int64_t n, hipStream_t st);

constexpr int kCellRec = 5;   // adjoint / stability cell records: nu, gamma, B_x, B_y, B_z

// power method of the stability estimate (eq. 8) on compact conducting-edge
// vectors (one block each): a unit start vector, and the normalisation of
// y = B v (lambda = ||y|| into *lam, v <- y / lambda, rec = {lambda, v^T y})
void power_init(int nc, double *v, hipStream_t st);
void power_norm(int nc, const double *y, double *v, double *lam, double *rec, hipStream_t st);

// discrete adjoint of the time loop (ec_adjoint.hip); the *part launchers
// return the number of block partials they wrote
void adj_cell_init(double *cellv, int64_t ncell, double nu0, hipStream_t st);
int adj_cell(const Geo &g, const Mats *mt, const uint8_t *cmat, const double *a, const double *w,
             double *cellv, int mat, const int lo[3], const int hi[3], double *part,
             hipStream_t st);
void adj_edge(const Geo &g, const int *cslot, int nc, const double *cellv, const double *u,
              double *out, hipStream_t st);
int adj_mu(int nc, const double *a_m, const double *a_m1, const double *mu_next, double *d_next,
           const double *minv, const double *phi, const double *jt, double dt, int terminal,
           double *mu_out, double *part, hipStream_t st);
void adj_w(const int *cslot, int nc, const double *mu, const double *minv, double *y,
           hipStream_t st);
int adj_loss(int nc, const double *a_new, const double *a_old, const double *minv, double dt,
             double *part, hipStream_t st);
void adj_accum(const double *part, int nb, double coef, double *acc, hipStream_t st);
void adj_zero(double *acc, int n, hipStream_t st);
void gather_c(const int *cslot, int nc, const double *src, double *dst, hipStream_t st);
void scatter_c(const int *cslot, int nc, const double *src, double *dst, hipStream_t st);

// the PCG solve of ec_solve_static (ec_capi.cpp) and what it needs to know
int64_t scratch_need(const ec_problem *h);
hipStream_t bound_stream(const ec_problem *h);
int32_t solve_scratch(ec_problem *h, int32_t method, const double *b, double *x,
                      const ec_solve_opts *o, ec_solve_info *info, char *scr, int64_t bytes,
                      hipError_t lookup);

// ----------------------------------------- consistent conductivity matrix
// M_c of the lowest-order edge elements on the compact conducting-edge list:
// at most kMassNnz entries per row, ELL columns idx/val[q * nc + e] (idx < 0:
// unused), dinv = 1 / diag (Jacobi)
constexpr int kMassNnz = 9;
struct MassOp {
    const int *idx;
    const double *val;
    const double *dinv;
    int nc;
};
// Jacobi-PCG of M_c y = b (compact vectors; single-reduction form, the
// record protocol of CgArgs): mode START_ZERO, or START_DEV (seq's start:
// zero_start, else x and rb[0] hold x0 and b - M x0)
struct MassCg {
    MassOp M;
    double *x;
    const double *b;
    double *p, *rb[2], *wb[2], *sb[2];
    CgCtl *ctl;              // [2]
    double *part;            // [2][kMaxBlocks][4]
    int blocks;
    double rtol;
    int maxit, mode;
    SeqDev *seq;
    ec_solve_info *info;     // may be nullptr
    Ctrl *ctrl;              // counters (may be nullptr)
};
int mass_blocks(int nc);
void mass_apply(const MassOp &M, const double *x, double *y, hipStream_t st);
void mass_cg_init(const MassCg &a, hipStream_t st);
void mass_cg_iter(const MassCg &a, int it, hipStream_t st);
void mass_cg_fin(const MassCg &a, int iters, hipStream_t st);
// SPE push slot product for the mass sequence (acceptance test in every block)
void mass_slots(const MassOp &M, int64_t ld, const double *x, double *ycopy, double *xcopy,
                double *ypen, const int *slot, SeqDev *sq, const double *pin, double tol,
                hipStream_t st);
void mass_axpy(const int *cslot, int nc, const double *A, const double *y, const Ctrl *ctrl,
               double *out, hipStream_t st);

// ------------------------------------------------ implicit Euler / Newton
// forward Jacobian: cell records (nu, d nu) of J_N(a) in direction v, and
// out = J_N(a) v - S v on the conducting edges from u = v (+) -K_n^+ K_cn^T v
void jn_cell(const Geo &g, const Mats *mt, const uint8_t *cmat, const double *a, const double *v,
             double *cellv, const int lo[3], const int hi[3], hipStream_t st);
void jn_edge(const Geo &g, const int *cslot, int nc, const double *cellv, const double *u,
             const double *a, double *out, hipStream_t st);
// GMRES(m) record: restart length at most kGmMax (its m + 1 basis columns fit
// the basis products' column limit kMaxWin)
constexpr int kGmMax = 20;
struct GmDev {
    int ncol, slot, conv, pad;
    double beta, target, res, a1;
    double H[(kGmMax + 1) * kGmMax];   // rotated Hessenberg matrix, row i at i * kGmMax
    double cs[kGmMax], sn[kGmMax], g[kGmMax + 1];
    double h1[kGmMax + 1], coef[kGmMax + 1];
};
int nrm2_part(int n, const double *x, double *part, hipStream_t st);
void nrm2_fin(const double *part, int nb, double *out, hipStream_t st);
void gm_begin(GmDev *gm, const double *part, int nb, int first, double rtol, hipStream_t st);
void gm_orth1(GmDev *gm, const double *part, int j, hipStream_t st);
void gm_orth2(GmDev *gm, const double *part, int j, hipStream_t st);
void gm_solve(GmDev *gm, int jn, hipStream_t st);
void gm_precond(int nc, const double *v, const double *jv, const double *minv, double dt,
                double *w, hipStream_t st);
void newton_residual(int nc, const int *cslot, const double *a, const double *a_old,
                     const double *minv, double dt, double *F, hipStream_t st);
void newton_update(int nc, const int *cslot, const double *d, double *a, hipStream_t st);
void vsub(int n, const double *x, const double *y, double *out, hipStream_t st);

}  // namespace ec
