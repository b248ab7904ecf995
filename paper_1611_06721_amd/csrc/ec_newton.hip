// ec_newton.hip -- the implicit Euler reference on gfx950 (the method the
// paper compares the semi-explicit scheme with, Secs. I and IV): Newton on
// the Schur form F(a) = M_c (a - a_old)/dt + N(a) - S a + K_cn K_n^+ j = 0,
// each Newton system J d = -F (J = M_c/dt + J_N(a) - S) solved by restarted
// GMRES, left-preconditioned by (M_c/dt)^-1 (then P^-1 J = I + dt M_c^-1
// (J_N - S)).  Compact conducting-edge vectors; the Arnoldi basis V holds
// columns ld apart and is orthogonalised by two classical Gram-Schmidt
// passes through the basis-product (MFMA) and combination kernels of
// ec_basis.hip; the Hessenberg columns, Givens rotations, residual estimate
// and back substitution run in one-block kernels on a device record.
#include "ec_device.h"

namespace ec {

// sum of squares of x[0..n) into per-block partials (grid of nb blocks)
__global__ void __launch_bounds__(256) k_nrm2_part(int n, const double *__restrict__ x,
                                                    double *part)
{
    double v[1] = {0.0};
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
        v[0] += x[e] * x[e];
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

int nrm2_part(int n, const double *x, double *part, hipStream_t st)
{
    const int nb = std::max(1, std::min((n + 255) / 256, 256));
    hipLaunchKernelGGL(k_nrm2_part, dim3(nb), dim3(256), 0, st, n, x, part);
    return nb;
}

// ||x|| from the partials into *out (one block, fixed order)
__global__ void k_nrm2_fin(const double *part, int nb, double *out)
{
    double s[1];
    reduce_partials<1>(part, nb, 1, s);
    if (threadIdx.x == 0) *out = sqrt(s[0]);
}

void nrm2_fin(const double *part, int nb, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_nrm2_fin, dim3(1), dim3(256), 0, st, part, nb, out);
}

// Start of a GMRES cycle on r (its |r|^2 partials in part): beta = ||r||,
// g = beta e_1, v_0 = r / beta (by the combination that follows: a1 = 1/beta,
// no columns, into column 0).  first: the target residual is rtol beta.
__global__ void k_gm_begin(GmDev *gm, const double *part, int nb, int first, double rtol)
{
    double s[1];
    reduce_partials<1>(part, nb, 1, s);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(s[0]);
    if (first) gm->target = rtol * beta;
    gm->beta = beta;
    gm->res = beta;
    for (int i = 0; i <= kGmMax; ++i) gm->g[i] = 0.0;
    gm->g[0] = beta;
    gm->a1 = beta > 0.0 ? 1.0 / beta : 0.0;
    gm->ncol = 0;
    gm->slot = 0;
    gm->conv = (beta <= gm->target || !(beta > 0.0)) ? 1 : 0;
}

// first Gram-Schmidt pass of column j: h1 = V_{0..j}^T w (reduced partial rows
// of the basis product), the combination w - V h1 follows
__global__ void k_gm_orth1(GmDev *gm, const double *part, int j)
{
    __shared__ double val[kMaxWin];
    reduce_rows<kMaxWin>(part, j + 1, j + 1, val);
    if (threadIdx.x <= j) {
        gm->h1[threadIdx.x] = val[threadIdx.x];
        gm->coef[threadIdx.x] = -val[threadIdx.x];
    }
    if (threadIdx.x == 0) {
        gm->a1 = 1.0;
        gm->ncol = j + 1;
    }
}

// second pass and the Hessenberg column j: h2 = V^T w' and |w'|^2 (partials of
// the combination), H[0..j][j] = h1 + h2, H[j+1][j] = ||w' - V h2|| (by
// Pythagoras), v_{j+1} = (w' - V h2) / H[j+1][j] by the combination that
// follows; the earlier Givens rotations on column j, a new one that zeroes
// H[j+1][j], g and the residual estimate |g_{j+1}|
__global__ void k_gm_orth2(GmDev *gm, const double *part, int j)
{
    __shared__ double val[kMaxWin];
    reduce_rows<kMaxWin>(part, kMaxWin, j + 2, val);
    if (threadIdx.x != 0) return;
    const int K = kGmMax;
    double nn = val[j + 1], h2s = 0.0;
    double col[kGmMax + 1];
    for (int i = 0; i <= j; ++i) {
        col[i] = gm->h1[i] + val[i];
        h2s += val[i] * val[i];
    }
    const double hn = sqrt(fmax(nn - h2s, 0.0));
    col[j + 1] = hn;
    for (int i = 0; i <= j + 1; ++i) gm->H[i * K + j] = col[i];
    for (int i = 0; i <= j; ++i) gm->coef[i] = hn > 0.0 ? -val[i] / hn : 0.0;
    gm->a1 = hn > 0.0 ? 1.0 / hn : 0.0;
    gm->ncol = j + 1;
    gm->slot = j + 1;
    // earlier rotations on the new column
    for (int i = 0; i < j; ++i) {
        const double t = gm->cs[i] * col[i] + gm->sn[i] * col[i + 1];
        col[i + 1] = -gm->sn[i] * col[i] + gm->cs[i] * col[i + 1];
        col[i] = t;
    }
    const double r = sqrt(col[j] * col[j] + col[j + 1] * col[j + 1]);
    const double c = r > 0.0 ? col[j] / r : 1.0, s = r > 0.0 ? col[j + 1] / r : 0.0;
    gm->cs[j] = c;
    gm->sn[j] = s;
    col[j] = r;
    col[j + 1] = 0.0;
    for (int i = 0; i <= j + 1; ++i) gm->H[i * K + j] = col[i];     // the rotated column
    const double gj = gm->g[j];
    gm->g[j] = c * gj;
    gm->g[j + 1] = -s * gj;
    gm->res = fabs(gm->g[j + 1]);
    gm->conv = (gm->res <= gm->target || !(hn > 1e-300 * (gm->beta + 1.0))) ? 1 : 0;
}

// back substitution of the rotated (upper triangular) H y = g on the first
// jn columns; coef = y for the update x += V y (combination that follows)
__global__ void k_gm_solve(GmDev *gm, int jn)
{
    if (threadIdx.x != 0) return;
    const int K = kGmMax;
    double y[kGmMax];
    for (int i = jn - 1; i >= 0; --i) {
        double t = gm->g[i];
        for (int q = i + 1; q < jn; ++q) t -= gm->H[i * K + q] * y[q];
        const double d = gm->H[i * K + i];
        y[i] = d != 0.0 ? t / d : 0.0;
    }
    for (int i = 0; i < jn; ++i) gm->coef[i] = y[i];
    gm->a1 = 1.0;
    gm->ncol = jn;
}

void gm_begin(GmDev *gm, const double *part, int nb, int first, double rtol, hipStream_t st)
{
    hipLaunchKernelGGL(k_gm_begin, dim3(1), dim3(256), 0, st, gm, part, nb, first, rtol);
}
void gm_orth1(GmDev *gm, const double *part, int j, hipStream_t st)
{
    hipLaunchKernelGGL(k_gm_orth1, dim3(1), dim3(kMdBlocks), 0, st, gm, part, j);
}
void gm_orth2(GmDev *gm, const double *part, int j, hipStream_t st)
{
    hipLaunchKernelGGL(k_gm_orth2, dim3(1), dim3(kMdBlocks), 0, st, gm, part, j);
}
void gm_solve(GmDev *gm, int jn, hipStream_t st)
{
    hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, st, gm, jn);
}

// w = v + dt minv (jv), the preconditioned product P^-1 J v from
// jv = (J_N - S) v; with neg: w = -dt minv jv (the right-hand side -P^-1 F)
__global__ void k_gm_precond(int nc, const double *__restrict__ v, const double *__restrict__ jv,
                             const double *__restrict__ minv, double dt, double *w)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc) return;
    w[e] = (v ? v[e] : 0.0) + (v ? dt : -dt) * minv[e] * jv[e];
}

void gm_precond(int nc, const double *v, const double *jv, const double *minv, double dt,
                double *w, hipStream_t st)
{
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_gm_precond, dim3((nc + 255) / 256), dim3(256), 0, st, nc, v, jv, minv,
                       dt, w);
}

// out = x - y (compact)
__global__ void k_sub(int n, const double *__restrict__ x, const double *__restrict__ y,
                      double *out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = x[e] - y[e];
}

void vsub(int n, const double *x, const double *y, double *out, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_sub, dim3((n + 255) / 256), dim3(256), 0, st, n, x, y, out);
}

// F = (a - a_old) / (dt minv) + g on the conducting edges (compact g, a read
// at the slots of the padded state a, a_old compact)
__global__ void k_newton_residual(int nc, const int *__restrict__ cslot,
                                  const double *__restrict__ a, const double *__restrict__ a_old,
                                  const double *__restrict__ minv, double dt, double *F)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc) return;
    F[e] = (a[cslot[e]] - a_old[e]) / (dt * minv[e]) + F[e];
}

void newton_residual(int nc, const int *cslot, const double *a, const double *a_old,
                     const double *minv, double dt, double *F, hipStream_t st)
{
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_newton_residual, dim3((nc + 255) / 256), dim3(256), 0, st, nc, cslot, a,
                       a_old, minv, dt, F);
}

// a += d at the conducting slots of the padded state
__global__ void k_newton_update(int nc, const int *__restrict__ cslot, const double *__restrict__ d,
                                double *a)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc) return;
    a[cslot[e]] += d[e];
}

void newton_update(int nc, const int *cslot, const double *d, double *a, hipStream_t st)
{
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_newton_update, dim3((nc + 255) / 256), dim3(256), 0, st, nc, cslot, d, a);
}

}  // namespace ec
