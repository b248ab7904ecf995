/*
 * ec_oracle.c -- plain FP64 CPU oracle of the semi-explicit eddy-current
 * scheme (Dutine, Clemens, Schoeps, "Multiple right-hand side techniques in
 * semi-explicit time integration methods for transient eddy current
 * problems").
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this file's library.  It shares no code, header or
 * table with the HIP library; the two agree only on the edge-array layout
 * documented in synth/__init__.py.
 *
 * What it computes, in the paper's terms:
 *   - the DAE blocks of eq. (3) on a staggered Cartesian (FIT) grid: the
 *     curl-curl operator K = C^T M_nu C restricted to non-Dirichlet edges and
 *     the diagonal conductivity matrix M_c = M_sigma (Sec. II);
 *   - the nonlinear reluctivity nu(|B|) of eq. (1) in conducting cells,
 *     here the Brauer curve nu = k1 exp(k2 |B|^2) + k3;
 *   - the pseudo-inverse K_n^+ b of eq. (9) by plain conjugate gradients from
 *     a zero start (Sec. III, weak gauging of Sec. II);
 *   - explicit Euler steps of the Schur-complement ODE, eqs. (5a), (6), (7),
 *     with the sign of eq. (5a) (derived from eq. (3));
 *   - the power method for the stability bound of eq. (8);
 *   - the discrete adjoint of the time loop (gradient of the Joule loss).
 *
 * Everything is written as plain loops over edges, faces and cells; no
 * blocking, fusion or reordering.  OpenMP only splits independent loop
 * iterations across threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { CLS_D = 0, CLS_C = 1, CLS_N = 2 };

typedef struct {
    int nx, ny, nz;
    double hx, hy, hz;
    long S;          /* entries per direction block: (nx+1)(ny+1)(nz+1) */
    long npad;       /* 3*S */
    long ncell;
    double nu0;
    int nmat;        /* number of materials incl. id 0 (nonconducting) */
    double *sig, *k1, *k2, *k3;
    uint8_t *cmat;   /* per cell material id */
    uint8_t *cls;    /* per edge class */
    double *msig;    /* per edge M_sigma (zero off C) */
    double *nu;      /* per cell reluctivity (scratch, set by nu_from) */
    double *face;    /* per face scratch, same padded layout as edges */
} orp;

/* ---------------------------------------------------------------- indexing */
static inline long EI(const orp *p, int c, long i, long j, long k)
{
    return (long)c * p->S + (k * (p->ny + 1) + j) * (p->nx + 1) + i;
}
static inline long CI(const orp *p, long i, long j, long k)
{
    return (k * p->ny + j) * p->nx + i;
}

/* --------------------------------------------------------------- threading */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ----------------------------------------------------------- create / free */
void or_destroy(void *h)
{
    orp *p = (orp *)h;
    if (!p) return;
    free(p->sig); free(p->k1); free(p->k2); free(p->k3);
    free(p->cmat); free(p->cls); free(p->msig); free(p->nu); free(p->face);
    free(p);
}

/*
 * Build the FIT problem.  cell_mat[c] = 0 marks a nonconducting cell with
 * reluctivity nu0; id m >= 1 selects material m-1 of the arrays (sigma, k1,
 * k2, k3).  Returns NULL on bad arguments.
 *
 * Edge classes (Sec. II, splitting of the dofs into a_c and a_n):
 *   D  edges tangential to the boundary (Dirichlet, removed) and padding;
 *   C  remaining edges with M_sigma > 0 (touching a conducting cell);
 *   N  the rest (nonconducting and source region).
 */
void *or_create(int nx, int ny, int nz, double lx, double ly, double lz,
                const uint8_t *cell_mat, int n_mats, const double *sig,
                const double *k1, const double *k2, const double *k3,
                double nu0)
{
    if (nx < 2 || ny < 2 || nz < 2 || n_mats < 0) return NULL;
    orp *p = (orp *)calloc(1, sizeof(orp));
    p->nx = nx; p->ny = ny; p->nz = nz;
    p->hx = lx / nx; p->hy = ly / ny; p->hz = lz / nz;
    p->S = (long)(nx + 1) * (ny + 1) * (nz + 1);
    p->npad = 3 * p->S;
    p->ncell = (long)nx * ny * nz;
    p->nu0 = nu0;
    p->nmat = n_mats + 1;
    p->sig = calloc(p->nmat, sizeof(double));
    p->k1 = calloc(p->nmat, sizeof(double));
    p->k2 = calloc(p->nmat, sizeof(double));
    p->k3 = calloc(p->nmat, sizeof(double));
    p->k3[0] = nu0;
    for (int m = 0; m < n_mats; ++m) {
        p->sig[m + 1] = sig[m]; p->k1[m + 1] = k1[m];
        p->k2[m + 1] = k2[m]; p->k3[m + 1] = k3[m];
    }
    p->cmat = malloc(p->ncell);
    for (long c = 0; c < p->ncell; ++c) {
        if (cell_mat[c] > n_mats) { or_destroy(p); return NULL; }
        p->cmat[c] = cell_mat[c];
    }
    p->cls = calloc(p->npad, 1);
    p->msig = calloc(p->npad, sizeof(double));
    p->nu = malloc(p->ncell * sizeof(double));
    p->face = calloc(p->npad, sizeof(double));

    /* M_sigma: each of the (up to) four cells around an edge contributes
     * sigma times a quarter of the dual face, divided by the edge length. */
    for (long k = 0; k <= nz; ++k)
    for (long j = 0; j <= ny; ++j)
    for (long i = 0; i <= nx; ++i) {
        /* x edge (i,j,k): cells (i, j-1..j, k-1..k) */
        if (i < nx) {
            double s = 0.0;
            for (long dj = -1; dj <= 0; ++dj) for (long dk = -1; dk <= 0; ++dk) {
                long jj = j + dj, kk = k + dk;
                if (jj >= 0 && jj < ny && kk >= 0 && kk < nz)
                    s += p->sig[p->cmat[CI(p, i, jj, kk)]];
            }
            long e = EI(p, 0, i, j, k);
            int interior = (j > 0 && j < ny && k > 0 && k < nz);
            p->msig[e] = interior ? s * (p->hy * p->hz / 4.0) / p->hx : 0.0;
            p->cls[e] = !interior ? CLS_D : (p->msig[e] > 0.0 ? CLS_C : CLS_N);
        }
        /* y edge (i,j,k): cells (i-1..i, j, k-1..k) */
        if (j < ny) {
            double s = 0.0;
            for (long di = -1; di <= 0; ++di) for (long dk = -1; dk <= 0; ++dk) {
                long ii = i + di, kk = k + dk;
                if (ii >= 0 && ii < nx && kk >= 0 && kk < nz)
                    s += p->sig[p->cmat[CI(p, ii, j, kk)]];
            }
            long e = EI(p, 1, i, j, k);
            int interior = (i > 0 && i < nx && k > 0 && k < nz);
            p->msig[e] = interior ? s * (p->hz * p->hx / 4.0) / p->hy : 0.0;
            p->cls[e] = !interior ? CLS_D : (p->msig[e] > 0.0 ? CLS_C : CLS_N);
        }
        /* z edge (i,j,k): cells (i-1..i, j-1..j, k) */
        if (k < nz) {
            double s = 0.0;
            for (long di = -1; di <= 0; ++di) for (long dj = -1; dj <= 0; ++dj) {
                long ii = i + di, jj = j + dj;
                if (ii >= 0 && ii < nx && jj >= 0 && jj < ny)
                    s += p->sig[p->cmat[CI(p, ii, jj, k)]];
            }
            long e = EI(p, 2, i, j, k);
            int interior = (i > 0 && i < nx && j > 0 && j < ny);
            p->msig[e] = interior ? s * (p->hx * p->hy / 4.0) / p->hz : 0.0;
            p->cls[e] = !interior ? CLS_D : (p->msig[e] > 0.0 ? CLS_C : CLS_N);
        }
    }
    for (long c = 0; c < p->ncell; ++c) p->nu[c] = p->k1[p->cmat[c]] + p->k3[p->cmat[c]];
    for (long c = 0; c < p->ncell; ++c) if (p->cmat[c] == 0) p->nu[c] = nu0;
    return p;
}

long or_npad(void *h) { return ((orp *)h)->npad; }
void or_edge_class(void *h, uint8_t *out) { orp *p = h; memcpy(out, p->cls, p->npad); }
void or_msigma(void *h, double *out) { orp *p = h; memcpy(out, p->msig, p->npad * sizeof(double)); }
void or_cell_nu(void *h, double *out) { orp *p = h; memcpy(out, p->nu, p->ncell * sizeof(double)); }

/* ------------------------------------------------------------------- curl */
/* b = C a: magnetic flux through every face (right-handed circulation). */
static void curl(const orp *p, const double *a, double *b)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    #pragma omp parallel for collapse(2) schedule(static)
    for (long k = 0; k <= nz; ++k)
    for (long j = 0; j <= ny; ++j)
    for (long i = 0; i <= nx; ++i) {
        /* x-normal face spanning y in [j,j+1], z in [k,k+1] */
        b[EI(p, 0, i, j, k)] = (j < ny && k < nz)
            ? a[EI(p, 1, i, j, k)] + a[EI(p, 2, i, j + 1, k)]
              - a[EI(p, 1, i, j, k + 1)] - a[EI(p, 2, i, j, k)] : 0.0;
        /* y-normal face spanning z in [k,k+1], x in [i,i+1] */
        b[EI(p, 1, i, j, k)] = (k < nz && i < nx)
            ? a[EI(p, 2, i, j, k)] + a[EI(p, 0, i, j, k + 1)]
              - a[EI(p, 2, i + 1, j, k)] - a[EI(p, 0, i, j, k)] : 0.0;
        /* z-normal face spanning x in [i,i+1], y in [j,j+1] */
        b[EI(p, 2, i, j, k)] = (i < nx && j < ny)
            ? a[EI(p, 0, i, j, k)] + a[EI(p, 1, i + 1, j, k)]
              - a[EI(p, 0, i, j + 1, k)] - a[EI(p, 1, i, j, k)] : 0.0;
    }
}

/* Cell flux density B: mean of the two opposite face fluxes over the area. */
static void cell_B(const orp *p, const double *b, long i, long j, long k, double B[3])
{
    B[0] = 0.5 * (b[EI(p, 0, i, j, k)] + b[EI(p, 0, i + 1, j, k)]) / (p->hy * p->hz);
    B[1] = 0.5 * (b[EI(p, 1, i, j, k)] + b[EI(p, 1, i, j + 1, k)]) / (p->hz * p->hx);
    B[2] = 0.5 * (b[EI(p, 2, i, j, k)] + b[EI(p, 2, i, j, k + 1)]) / (p->hx * p->hy);
}

/* Reluctivity per cell from the state v: Brauer curve in material cells. */
static void nu_from(orp *p, const double *v)
{
    curl(p, v, p->face);
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    #pragma omp parallel for collapse(2) schedule(static)
    for (long k = 0; k < nz; ++k)
    for (long j = 0; j < ny; ++j)
    for (long i = 0; i < nx; ++i) {
        long c = CI(p, i, j, k);
        int m = p->cmat[c];
        if (m == 0) { p->nu[c] = p->nu0; continue; }
        double B[3];
        cell_B(p, p->face, i, j, k, B);
        double s = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
        p->nu[c] = p->k1[m] * exp(p->k2[m] * s) + p->k3[m];
    }
}

/* Face reluctance M_nu,f: mean of the two adjacent cells' nu times
 * (dual edge length / face area).  Boundary faces touch Dirichlet edges only;
 * they get the single adjacent cell's value. */
static double face_w(const orp *p, int c, long i, long j, long k)
{
    double nu_a, nu_b;
    if (c == 0) {
        long i0 = i > 0 ? i - 1 : i, i1 = i < p->nx ? i : i - 1;
        nu_a = p->nu[CI(p, i0, j, k)]; nu_b = p->nu[CI(p, i1, j, k)];
        return 0.5 * (nu_a + nu_b) * p->hx / (p->hy * p->hz);
    } else if (c == 1) {
        long j0 = j > 0 ? j - 1 : j, j1 = j < p->ny ? j : j - 1;
        nu_a = p->nu[CI(p, i, j0, k)]; nu_b = p->nu[CI(p, i, j1, k)];
        return 0.5 * (nu_a + nu_b) * p->hy / (p->hz * p->hx);
    } else {
        long k0 = k > 0 ? k - 1 : k, k1 = k < p->nz ? k : k - 1;
        nu_a = p->nu[CI(p, i, j, k0)]; nu_b = p->nu[CI(p, i, j, k1)];
        return 0.5 * (nu_a + nu_b) * p->hz / (p->hx * p->hy);
    }
}

/* y = C^T M_nu C x on every non-Dirichlet edge (zero on D), using the
 * reluctivity currently stored in p->nu. */
static void apply_K(orp *p, const double *x, double *y)
{
    double *hf = p->face;
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    curl(p, x, hf);
    #pragma omp parallel for collapse(2) schedule(static)
    for (long k = 0; k <= nz; ++k)
    for (long j = 0; j <= ny; ++j)
    for (long i = 0; i <= nx; ++i) {
        if (j < ny && k < nz) hf[EI(p, 0, i, j, k)] *= face_w(p, 0, i, j, k);
        if (k < nz && i < nx) hf[EI(p, 1, i, j, k)] *= face_w(p, 1, i, j, k);
        if (i < nx && j < ny) hf[EI(p, 2, i, j, k)] *= face_w(p, 2, i, j, k);
    }
    /* C^T: every edge collects its four faces with the circulation signs. */
    #pragma omp parallel for collapse(2) schedule(static)
    for (long k = 0; k <= nz; ++k)
    for (long j = 0; j <= ny; ++j)
    for (long i = 0; i <= nx; ++i) {
        long ex = EI(p, 0, i, j, k), ey = EI(p, 1, i, j, k), ez = EI(p, 2, i, j, k);
        y[ex] = (p->cls[ex] == CLS_D) ? 0.0
              : hf[EI(p, 2, i, j, k)] - hf[EI(p, 2, i, j - 1, k)]
                - hf[EI(p, 1, i, j, k)] + hf[EI(p, 1, i, j, k - 1)];
        y[ey] = (p->cls[ey] == CLS_D) ? 0.0
              : hf[EI(p, 0, i, j, k)] - hf[EI(p, 0, i, j, k - 1)]
                - hf[EI(p, 2, i, j, k)] + hf[EI(p, 2, i - 1, j, k)];
        y[ez] = (p->cls[ez] == CLS_D) ? 0.0
              : hf[EI(p, 1, i, j, k)] - hf[EI(p, 1, i - 1, j, k)]
                - hf[EI(p, 0, i, j, k)] + hf[EI(p, 0, i, j - 1, k)];
    }
}

/* Public: y = K x with nu taken from state v (v may equal x). */
void or_apply(void *h, const double *v, const double *x, double *y)
{
    orp *p = h;
    nu_from(p, v);
    apply_K(p, x, y);
}

/* Public: per-cell B (3 per cell, cell index major) of state v. */
void or_cell_B(void *h, const double *v, double *B)
{
    orp *p = h;
    curl(p, v, p->face);
    for (long k = 0; k < p->nz; ++k)
    for (long j = 0; j < p->ny; ++j)
    for (long i = 0; i < p->nx; ++i)
        cell_B(p, p->face, i, j, k, B + 3 * CI(p, i, j, k));
}

/* Public: face fluxes b = C a (padded layout). */
void or_curl(void *h, const double *a, double *b) { curl((orp *)h, a, b); }

static void mask(const orp *p, double *v, int cls)
{
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < p->npad; ++e) if (p->cls[e] != cls) v[e] = 0.0;
}

/* K_n x = [K (x restricted to N)]_N.  Faces touching an N edge are air, so
 * the reluctivity in conducting cells does not enter. */
static void apply_Kn(orp *p, const double *x, double *y, double *tmp)
{
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < p->npad; ++e) tmp[e] = p->cls[e] == CLS_N ? x[e] : 0.0;
    apply_K(p, tmp, y);
    mask(p, y, CLS_N);
}
void or_kn(void *h, const double *x, double *y)
{
    orp *p = h;
    double *t = malloc(p->npad * sizeof(double));
    apply_Kn(p, x, y, t);
    free(t);
}

/* K_cn^T a_c = [K (a restricted to C)]_N. */
static void apply_KcnT(orp *p, const double *a, double *y, double *tmp)
{
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < p->npad; ++e) tmp[e] = p->cls[e] == CLS_C ? a[e] : 0.0;
    apply_K(p, tmp, y);
    mask(p, y, CLS_N);
}
void or_kcnT(void *h, const double *a, double *y)
{
    orp *p = h;
    double *t = malloc(p->npad * sizeof(double));
    apply_KcnT(p, a, y, t);
    free(t);
}

static double dot(long n, const double *a, const double *b)
{
    double s = 0.0;
    #pragma omp parallel for reduction(+:s) schedule(static)
    for (long e = 0; e < n; ++e) s += a[e] * b[e];
    return s;
}

/* ------------------------------------------------------------------- CG */
/*
 * Conjugate gradients for K_n x = b (eq. 9), started from the given x.
 * Stops when ||b - K_n x||_2 <= rtol ||b||_2 (recursive residual).  b = 0
 * returns x = 0 after 0 iterations.  Returns 0, or -3 when maxit is reached,
 * -4 on breakdown (p^T K p <= 0 with r != 0).
 */
static int cg(orp *p, const double *b, double *x, double rtol, int maxit,
              int *iters, double *relres, double *r, double *pp, double *q, double *tmp)
{
    long n = p->npad;
    double bb = dot(n, b, b);
    *iters = 0;
    if (bb == 0.0) {
        memset(x, 0, n * sizeof(double));
        *relres = 0.0;
        return 0;
    }
    apply_Kn(p, x, q, tmp);
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < n; ++e) { r[e] = b[e] - q[e]; pp[e] = r[e]; }
    double rr = dot(n, r, r);
    double tol2 = rtol * rtol * bb;
    int it = 0, st = 0;
    while (rr > tol2) {
        if (it >= maxit) { st = -3; break; }
        apply_Kn(p, pp, q, tmp);
        double pq = dot(n, pp, q);
        if (!(pq > 0.0)) { st = -4; break; }
        double alpha = rr / pq;
        #pragma omp parallel for schedule(static)
        for (long e = 0; e < n; ++e) { x[e] += alpha * pp[e]; r[e] -= alpha * q[e]; }
        double rr_new = dot(n, r, r);
        double beta = rr_new / rr;
        #pragma omp parallel for schedule(static)
        for (long e = 0; e < n; ++e) pp[e] = r[e] + beta * pp[e];
        rr = rr_new;
        ++it;
    }
    *iters = it;
    *relres = sqrt(rr / bb);
    return st;
}

int or_cg(void *h, const double *b, double *x, double rtol, int maxit,
          int *iters, double *relres)
{
    orp *p = h;
    long n = p->npad;
    double *w = malloc(4 * n * sizeof(double));
    int st = cg(p, b, x, rtol, maxit, iters, relres, w, w + n, w + 2 * n, w + 3 * n);
    free(w);
    return st;
}

/* ------------------------------------------------------------- waveform */
/* i_S at step m (t = m dt): 0 DC, 1 sine, 2 linear ramp over ramp_steps,
 * 3 the 1 - exp(-t/tau) excitation of the paper's benchmark (Sec. IV). */
double or_waveform(int wf, double amp, double freq, double tau, long ramp_steps,
                   long m, double dt)
{
    double t = m * dt;
    switch (wf) {
    case 0: return amp;
    case 1: return amp * sin(2.0 * M_PI * freq * t);
    case 2: return amp * (m >= ramp_steps ? 1.0 : (double)m / (double)ramp_steps);
    case 3: return amp * (1.0 - exp(-t / tau));
    default: return 0.0;
    }
}

/* --------------------------------------------------------- explicit Euler */
typedef struct {
    double *sj, *sc, *b, *v, *g, *r, *pp, *q, *tmp;
} work_t;

static work_t work_alloc(long n)
{
    work_t w;
    double *blk = calloc(9 * n, sizeof(double));
    w.sj = blk; w.sc = blk + n; w.b = blk + 2 * n; w.v = blk + 3 * n;
    w.g = blk + 4 * n; w.r = blk + 5 * n; w.pp = blk + 6 * n; w.q = blk + 7 * n;
    w.tmp = blk + 8 * n;
    return w;
}

/*
 * One explicit Euler step m (eqs. 6 and 7 with the sign of eq. 5a):
 *   s_j   = K_n^+ j^m                       (j^m = i_S(t_m) X_S)
 *   y     = s_j - s_c                        (s_c = K_n^+ K_cn^T a_c^{m-1})
 *   g     = K_c(a_c^{m-1}) a_c^{m-1} + K_cn y
 *   a_c^m = a_c^{m-1} - dt M_c^{-1} g
 *   s_c   = K_n^+ K_cn^T a_c^m
 *   a_n^m = s_j - s_c
 * A holds a_c on C edges and a_n on N edges; sc carries s_c between steps.
 */
static int step(orp *p, work_t *w, double *A, const double *xs, double isrc,
                double dt, double rtol, int maxit, int *it_src, int *it_cpl)
{
    long n = p->npad;
    double rel;
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < n; ++e) { w->b[e] = isrc * xs[e]; w->sj[e] = 0.0; }
    mask(p, w->b, CLS_N);
    int st = cg(p, w->b, w->sj, rtol, maxit, it_src, &rel, w->r, w->pp, w->q, w->tmp);
    if (st) return st;
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < n; ++e)
        w->v[e] = p->cls[e] == CLS_C ? A[e] : (p->cls[e] == CLS_N ? w->sj[e] - w->sc[e] : 0.0);
    nu_from(p, w->v);                       /* nu(a_c^{m-1}) */
    apply_K(p, w->v, w->g);
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < n; ++e)
        if (p->cls[e] == CLS_C) A[e] -= dt * w->g[e] / p->msig[e];
    apply_KcnT(p, A, w->b, w->tmp);
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < n; ++e) w->sc[e] = 0.0;
    st = cg(p, w->b, w->sc, rtol, maxit, it_cpl, &rel, w->r, w->pp, w->q, w->tmp);
    if (st) return st;
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < n; ++e)
        if (p->cls[e] == CLS_N) A[e] = w->sj[e] - w->sc[e];
    return 0;
}

/*
 * Run steps m0+1 .. m0+nsteps from state A (in/out).  sc (in/out, may be
 * NULL for a zero start) carries K_n^+ K_cn^T a_c between calls.  Every
 * rec_every steps A is appended to rec (if rec != NULL).  Per-step iteration
 * counts go to it_src / it_cpl when given.  Returns 0 or the CG status.
 */
int or_run(void *h, double *A, double *sc, const double *xs, int wf, double amp,
           double freq, double tau, long ramp_steps, double dt, long m0, long nsteps,
           double rtol, int maxit, long rec_every, double *rec,
           int *it_src, int *it_cpl)
{
    orp *p = h;
    long n = p->npad;
    work_t w = work_alloc(n);
    if (sc) memcpy(w.sc, sc, n * sizeof(double));
    int st = 0;
    long nrec = 0;
    for (long s = 1; s <= nsteps; ++s) {
        long m = m0 + s;
        double isrc = or_waveform(wf, amp, freq, tau, ramp_steps, m, dt);
        int a = 0, b = 0;
        st = step(p, &w, A, xs, isrc, dt, rtol, maxit, &a, &b);
        if (it_src) it_src[s - 1] = a;
        if (it_cpl) it_cpl[s - 1] = b;
        if (st) break;
        if (rec && rec_every > 0 && s % rec_every == 0)
            memcpy(rec + (nrec++) * n, A, n * sizeof(double));
    }
    if (sc) memcpy(sc, w.sc, n * sizeof(double));
    free(w.sj);
    return st;
}

/* ------------------------------------------------------ stability bound */
/*
 * Largest eigenvalue of M_c^{-1} K_S(a_c) (eq. 8) by the power method, with
 * the reluctivity frozen at state A.  K_S v = [K (v (+) -K_n^+ K_cn^T v)]_C.
 * The iteration runs in the M_c inner product, where M_c^{-1} K_S is
 * self-adjoint; the estimate is the Rayleigh quotient v^T K_S v / v^T M_c v.
 */
double or_power(void *h, const double *A, int iters, double rtol, unsigned seed)
{
    orp *p = h;
    long n = p->npad;
    work_t w = work_alloc(n);
    double *vc = malloc(n * sizeof(double));
    double *Ks = malloc(n * sizeof(double));
    nu_from(p, A);
    double *nu_frozen = malloc(p->ncell * sizeof(double));
    memcpy(nu_frozen, p->nu, p->ncell * sizeof(double));
    unsigned s = seed ? seed : 12345u;
    for (long e = 0; e < n; ++e) {
        s = s * 1664525u + 1013904223u;
        vc[e] = p->cls[e] == CLS_C ? ((double)(s >> 8) / 16777216.0 - 0.5) : 0.0;
    }
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        double nrm = 0.0;
        for (long e = 0; e < n; ++e) if (p->cls[e] == CLS_C) nrm += vc[e] * vc[e] * p->msig[e];
        nrm = sqrt(nrm);
        for (long e = 0; e < n; ++e) vc[e] /= nrm;
        /* s = K_n^+ K_cn^T v */
        memcpy(p->nu, nu_frozen, p->ncell * sizeof(double));
        apply_KcnT(p, vc, w.b, w.tmp);
        memset(w.sc, 0, n * sizeof(double));
        int ci; double rel;
        cg(p, w.b, w.sc, rtol, 100000, &ci, &rel, w.r, w.pp, w.q, w.tmp);
        for (long e = 0; e < n; ++e)
            w.v[e] = p->cls[e] == CLS_C ? vc[e] : (p->cls[e] == CLS_N ? -w.sc[e] : 0.0);
        memcpy(p->nu, nu_frozen, p->ncell * sizeof(double));
        apply_K(p, w.v, Ks);
        double num = 0.0;
        for (long e = 0; e < n; ++e) if (p->cls[e] == CLS_C) num += vc[e] * Ks[e];
        lam = num;   /* v is M_c-normalised */
        for (long e = 0; e < n; ++e) vc[e] = p->cls[e] == CLS_C ? Ks[e] / p->msig[e] : 0.0;
    }
    free(vc); free(Ks); free(nu_frozen); free(w.sj);
    return lam;
}

/* ------------------------------------------------------------- adjoint */
/*
 * Pieces of the discrete adjoint of the time loop.  With the conducting
 * block N(a) = [C^T M_nu(a) C a]_C (a on C edges, the reluctivity of the iron
 * cells taken from a through their cell B), one step is
 *   F(a) = a - dt M_c^{-1} [ N(a) - S a + K_cn K_n^+ j ],  S = K_cn K_n^+ K_cn^T,
 * and the adjoint needs J_N(a)^T, dN/dk1 and dM_c/dsigma.  J_N is not
 * symmetric (face-averaged nu), so its transpose is written out.
 */

/* geometric part of the face reluctance: dual edge length / face area */
static double face_geo(const orp *p, int c)
{
    if (c == 0) return p->hx / (p->hy * p->hz);
    if (c == 1) return p->hy / (p->hz * p->hx);
    return p->hz / (p->hx * p->hy);
}

static double face_area(const orp *p, int c)
{
    if (c == 0) return p->hy * p->hz;
    if (c == 1) return p->hz * p->hx;
    return p->hx * p->hy;
}

/* does face (c,i,j,k) exist, and the two cells whose nu it averages */
static int face_cells(const orp *p, int c, long i, long j, long k, long *ca, long *cb)
{
    if (c == 0) {
        if (!(j < p->ny && k < p->nz)) return 0;
        long i0 = i > 0 ? i - 1 : i, i1 = i < p->nx ? i : i - 1;
        *ca = CI(p, i0, j, k); *cb = CI(p, i1, j, k);
    } else if (c == 1) {
        if (!(k < p->nz && i < p->nx)) return 0;
        long j0 = j > 0 ? j - 1 : j, j1 = j < p->ny ? j : j - 1;
        *ca = CI(p, i, j0, k); *cb = CI(p, i, j1, k);
    } else {
        if (!(i < p->nx && j < p->ny)) return 0;
        long k0 = k > 0 ? k - 1 : k, k1 = k < p->nz ? k : k - 1;
        *ca = CI(p, i, j, k0); *cb = CI(p, i, j, k1);
    }
    return 1;
}

/* y = C^T f on every edge, then restricted to C edges */
static void curlT_c(const orp *p, const double *hf, double *y)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    for (long k = 0; k <= nz; ++k)
    for (long j = 0; j <= ny; ++j)
    for (long i = 0; i <= nx; ++i) {
        long ex = EI(p, 0, i, j, k), ey = EI(p, 1, i, j, k), ez = EI(p, 2, i, j, k);
        y[ex] = (p->cls[ex] != CLS_C) ? 0.0
              : hf[EI(p, 2, i, j, k)] - hf[EI(p, 2, i, j - 1, k)]
                - hf[EI(p, 1, i, j, k)] + hf[EI(p, 1, i, j, k - 1)];
        y[ey] = (p->cls[ey] != CLS_C) ? 0.0
              : hf[EI(p, 0, i, j, k)] - hf[EI(p, 0, i, j, k - 1)]
                - hf[EI(p, 2, i, j, k)] + hf[EI(p, 2, i - 1, j, k)];
        y[ez] = (p->cls[ez] != CLS_C) ? 0.0
              : hf[EI(p, 1, i, j, k)] - hf[EI(p, 1, i - 1, j, k)]
                - hf[EI(p, 0, i, j, k)] + hf[EI(p, 0, i, j - 1, k)];
    }
}

/* the C-edge part of a (zero elsewhere) */
static double *c_part(const orp *p, const double *a)
{
    double *o = malloc(p->npad * sizeof(double));
    for (long e = 0; e < p->npad; ++e) o[e] = p->cls[e] == CLS_C ? a[e] : 0.0;
    return o;
}

/* dnu/ds of cell c at s = |B|^2 (Brauer: k1 k2 exp(k2 s)) */
static double dnu_ds(const orp *p, long c, double s)
{
    int m = p->cmat[c];
    if (m == 0) return 0.0;
    return p->k1[m] * p->k2[m] * exp(p->k2[m] * s);
}

/* y = J_N(a) v on C edges: the derivative of N along v (a, v read on C). */
void or_jn(void *h, const double *a, const double *v, double *y)
{
    orp *p = h;
    const long n = p->npad;
    double *ac = c_part(p, a), *vc = c_part(p, v);
    double *fa = malloc(n * sizeof(double)), *fv = malloc(n * sizeof(double));
    double *hf = calloc(n, sizeof(double)), *dnu = calloc(p->ncell, sizeof(double));
    nu_from(p, ac);
    curl(p, ac, fa);
    curl(p, vc, fv);
    for (long k = 0; k < p->nz; ++k)
    for (long j = 0; j < p->ny; ++j)
    for (long i = 0; i < p->nx; ++i) {
        long c = CI(p, i, j, k);
        if (p->cmat[c] == 0) continue;
        double B[3], dB[3];
        cell_B(p, fa, i, j, k, B);
        cell_B(p, fv, i, j, k, dB);
        double s = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
        dnu[c] = dnu_ds(p, c, s) * 2.0 * (B[0] * dB[0] + B[1] * dB[1] + B[2] * dB[2]);
    }
    for (int d = 0; d < 3; ++d)
    for (long k = 0; k <= p->nz; ++k)
    for (long j = 0; j <= p->ny; ++j)
    for (long i = 0; i <= p->nx; ++i) {
        long ca, cb;
        if (!face_cells(p, d, i, j, k, &ca, &cb)) continue;
        long f = EI(p, d, i, j, k);
        hf[f] = face_w(p, d, i, j, k) * fv[f]
              + face_geo(p, d) * 0.5 * (dnu[ca] + dnu[cb]) * fa[f];
    }
    curlT_c(p, hf, y);
    free(ac); free(vc); free(fa); free(fv); free(hf); free(dnu);
}

/* y = J_N(a)^T lam on C edges (a, lam read on C). */
void or_jnT(void *h, const double *a, const double *lam, double *y)
{
    orp *p = h;
    const long n = p->npad;
    double *ac = c_part(p, a), *lc = c_part(p, lam);
    double *fa = malloc(n * sizeof(double)), *fl = malloc(n * sizeof(double));
    double *hf = calloc(n, sizeof(double));
    double *acc = calloc(p->ncell, sizeof(double));
    nu_from(p, ac);
    curl(p, ac, fa);
    curl(p, lc, fl);
    /* acc_c = sum over the (face, side) pairs with side cell c of w_f (C lam)_f (C a)_f */
    for (int d = 0; d < 3; ++d)
    for (long k = 0; k <= p->nz; ++k)
    for (long j = 0; j <= p->ny; ++j)
    for (long i = 0; i <= p->nx; ++i) {
        long ca, cb;
        if (!face_cells(p, d, i, j, k, &ca, &cb)) continue;
        long f = EI(p, d, i, j, k);
        double t = face_geo(p, d) * fl[f] * fa[f];
        acc[ca] += t;
        acc[cb] += t;
    }
    /* gamma_c = nu'(s_c) acc_c; q on the six faces of c: gamma_c B_c[dir] / (2 area) */
    for (long k = 0; k < p->nz; ++k)
    for (long j = 0; j < p->ny; ++j)
    for (long i = 0; i < p->nx; ++i) {
        long c = CI(p, i, j, k);
        if (p->cmat[c] == 0) continue;
        double B[3];
        cell_B(p, fa, i, j, k, B);
        double s = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
        double g = dnu_ds(p, c, s) * acc[c];
        if (g == 0.0) continue;
        hf[EI(p, 0, i, j, k)] += g * 0.5 * B[0] / face_area(p, 0);
        hf[EI(p, 0, i + 1, j, k)] += g * 0.5 * B[0] / face_area(p, 0);
        hf[EI(p, 1, i, j, k)] += g * 0.5 * B[1] / face_area(p, 1);
        hf[EI(p, 1, i, j + 1, k)] += g * 0.5 * B[1] / face_area(p, 1);
        hf[EI(p, 2, i, j, k)] += g * 0.5 * B[2] / face_area(p, 2);
        hf[EI(p, 2, i, j, k + 1)] += g * 0.5 * B[2] / face_area(p, 2);
    }
    /* plus the symmetric part M_nu C lam */
    for (int d = 0; d < 3; ++d)
    for (long k = 0; k <= p->nz; ++k)
    for (long j = 0; j <= p->ny; ++j)
    for (long i = 0; i <= p->nx; ++i) {
        long ca, cb;
        if (!face_cells(p, d, i, j, k, &ca, &cb)) continue;
        long f = EI(p, d, i, j, k);
        hf[f] += face_w(p, d, i, j, k) * fl[f];
    }
    curlT_c(p, hf, y);
    free(ac); free(lc); free(fa); free(fl); free(hf); free(acc);
}

/* y = dN/dk1 of material mat at a (on C edges): C^T diag(dM_nu/dk1) C a with
 * dM_nu,f/dk1 = w_f * mean over the face's two cells of exp(k2 s_c)
 * (cells of material mat; zero for the others). */
void or_dn_dk1(void *h, const double *a, int mat, double *y)
{
    orp *p = h;
    const long n = p->npad;
    double *ac = c_part(p, a);
    double *fa = malloc(n * sizeof(double)), *hf = calloc(n, sizeof(double));
    double *e = calloc(p->ncell, sizeof(double));
    curl(p, ac, fa);
    for (long k = 0; k < p->nz; ++k)
    for (long j = 0; j < p->ny; ++j)
    for (long i = 0; i < p->nx; ++i) {
        long c = CI(p, i, j, k);
        if (p->cmat[c] != mat || mat == 0) continue;
        double B[3];
        cell_B(p, fa, i, j, k, B);
        e[c] = exp(p->k2[mat] * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]));
    }
    for (int d = 0; d < 3; ++d)
    for (long k = 0; k <= p->nz; ++k)
    for (long j = 0; j <= p->ny; ++j)
    for (long i = 0; i <= p->nx; ++i) {
        long ca, cb;
        if (!face_cells(p, d, i, j, k, &ca, &cb)) continue;
        long f = EI(p, d, i, j, k);
        hf[f] = face_geo(p, d) * 0.5 * (e[ca] + e[cb]) * fa[f];
    }
    curlT_c(p, hf, y);
    free(ac); free(fa); free(hf); free(e);
}

/* dM_sigma/dsigma of material mat on every edge (zero off C): the quarter
 * dual faces of the edge's cells of that material over the edge length. */
void or_dmsig(void *h, int mat, double *y)
{
    orp *p = h;
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    memset(y, 0, p->npad * sizeof(double));
    for (long k = 0; k <= nz; ++k)
    for (long j = 0; j <= ny; ++j)
    for (long i = 0; i <= nx; ++i) {
        if (i < nx && p->cls[EI(p, 0, i, j, k)] == CLS_C) {
            int cnt = 0;
            for (long dj = -1; dj <= 0; ++dj) for (long dk = -1; dk <= 0; ++dk)
                cnt += p->cmat[CI(p, i, j + dj, k + dk)] == mat;
            y[EI(p, 0, i, j, k)] = cnt * (p->hy * p->hz / 4.0) / p->hx;
        }
        if (j < ny && p->cls[EI(p, 1, i, j, k)] == CLS_C) {
            int cnt = 0;
            for (long di = -1; di <= 0; ++di) for (long dk = -1; dk <= 0; ++dk)
                cnt += p->cmat[CI(p, i + di, j, k + dk)] == mat;
            y[EI(p, 1, i, j, k)] = cnt * (p->hz * p->hx / 4.0) / p->hy;
        }
        if (k < nz && p->cls[EI(p, 2, i, j, k)] == CLS_C) {
            int cnt = 0;
            for (long di = -1; di <= 0; ++di) for (long dj = -1; dj <= 0; ++dj)
                cnt += p->cmat[CI(p, i + di, j + dj, k)] == mat;
            y[EI(p, 2, i, j, k)] = cnt * (p->hx * p->hy / 4.0) / p->hz;
        }
    }
}
