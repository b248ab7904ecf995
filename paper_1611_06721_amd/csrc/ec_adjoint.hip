// ec_adjoint.hip -- discrete adjoint of the explicit Euler loop on gfx950.
//
// One step (eqs. 6-7 with the sign of eq. 5a) maps the conducting unknowns
//   a^m = a^{m-1} - dt M_c^{-1} [ N(a^{m-1}) - S a^{m-1} + K_cn K_n^+ j^m ],
// N(a) = [C^T M_nu(a) C a]_C with the Brauer reluctivity of eq. (1) in the
// iron cells, S = K_cn K_n^+ K_cn^T.  For the Joule loss
//   L = sum_m (1/dt) d_m^T M_c d_m,  d_m = a^m - a^{m-1},
// the adjoint mu_m = dL/da^m obeys
//   mu_m = (2/dt) M_c (d_m - d_{m+1}) + mu_{m+1} - dt [J_N(a^m)^T - S] w,
//   w = M_c^{-1} mu_{m+1},
// and the gradients are
//   dL/dsigma = sum_m [ (1/dt) d_m^T Phi d_m - mu_m^T M_c^{-1} Phi d_m ],
//   dL/dk1    = -dt sum_m w_m^T dN/dk1(a^{m-1}),
// Phi = dM_c/dsigma.  J_N^T w = [C^T (M_nu C w + q)]_C with, per iron cell,
// gamma_c = nu'(s_c) sum_{faces f of c} g_f (Cw)_f (Ca)_f  (g_f = dual edge /
// face area, s_c = |B_c|^2) and q_f = sum_{cells c of f} gamma_c B_c,n / (2 A_f).
// The k1 term needs no edge pass: w^T dN/dk1(a) = 1/2 sum_c e^{k2 s_c} acc_c.
//
// Vectors on conducting edges are compact (slot list order); a, w and u are
// padded edge arrays whose nonconducting part is zero (a, w) or -K_n^+ K_cn^T w (u).
#include "ec_device.h"

namespace ec {


// flux of x through the face with normal n anchored at node (i, j, k)
// (right-handed circulation, same orientation as the curl-curl stencil)
__device__ __forceinline__ double face_flux(const Geo &g, const double *__restrict__ x, int n,
                                            int i, int j, int k)
{
    const int64_t off[3] = {1, g.px, (int64_t)g.px * g.py};
    const int64_t node = (int64_t)k * off[2] + (int64_t)j * off[1] + i;
    const int n1 = n == 2 ? 0 : n + 1, n2 = n == 0 ? 2 : n - 1;
    const double *x1 = x + (int64_t)n1 * g.S, *x2 = x + (int64_t)n2 * g.S;
    return x1[node] + x2[node + off[n1]] - x1[node + off[n2]] - x2[node];
}

__device__ __forceinline__ double face_geo(const Geo &g, int n)
{
    return n == 0 ? g.hx / (g.hy * g.hz) : (n == 1 ? g.hy / (g.hz * g.hx) : g.hz / (g.hx * g.hy));
}

__device__ __forceinline__ double face_area(const Geo &g, int n)
{
    return n == 0 ? g.hy * g.hz : (n == 1 ? g.hz * g.hx : g.hx * g.hy);
}

// air defaults of the cell records (conducting cells are rewritten per step)
__global__ void k_adj_cell_init(double *cellv, int64_t ncell, double nu0)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    cellv[c * kCellRec + 0] = nu0;
#pragma unroll
    for (int q = 1; q < kCellRec; ++q) cellv[c * kCellRec + q] = 0.0;
}

// Cell pass over the conductor's bounding box: nu, gamma, B of every
// conducting cell at state a for the adjoint direction w, and per block the
// partial sum of 1/2 e^{k2 s} acc over cells of material `mat`.
__global__ void __launch_bounds__(256)
    k_adj_cell(Geo g, const Mats *__restrict__ mt, const uint8_t *__restrict__ cmat,
               const double *__restrict__ a, const double *__restrict__ w, double *cellv,
               int mat, int lo0, int lo1, int lo2, int ex, int ey, int ez, double *part)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cnt = (int64_t)ex * ey * ez;
    double v[1] = {0.0};
    if (t < cnt) {
        const int64_t exy = (int64_t)ex * ey;
        const int kk = (int)(t / exy);
        const int64_t rem = t - (int64_t)kk * exy;
        const int jj = (int)(rem / ex), ii = (int)(rem - (int64_t)jj * ex);
        const int i = ii + lo0, j = jj + lo1, k = kk + lo2;
        const int64_t c = ((int64_t)k * g.ny + j) * g.nx + i;
        const int m = cmat[c];
        if (m) {
            const double fa[6] = {face_flux(g, a, 0, i, j, k), face_flux(g, a, 0, i + 1, j, k),
                                  face_flux(g, a, 1, i, j, k), face_flux(g, a, 1, i, j + 1, k),
                                  face_flux(g, a, 2, i, j, k), face_flux(g, a, 2, i, j, k + 1)};
            // no direction (w = nullptr): gamma = 0, the records of the
            // secant operator K_c(nu(a))
            double fw[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (w) {
                fw[0] = face_flux(g, w, 0, i, j, k); fw[1] = face_flux(g, w, 0, i + 1, j, k);
                fw[2] = face_flux(g, w, 1, i, j, k); fw[3] = face_flux(g, w, 1, i, j + 1, k);
                fw[4] = face_flux(g, w, 2, i, j, k); fw[5] = face_flux(g, w, 2, i, j, k + 1);
            }
            const double B[3] = {0.5 * (fa[0] + fa[1]) / face_area(g, 0),
                                 0.5 * (fa[2] + fa[3]) / face_area(g, 1),
                                 0.5 * (fa[4] + fa[5]) / face_area(g, 2)};
            const double s = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
            const double e = exp(mt->k2[m] * s);
            const double nu = mt->k1[m] * e + mt->k3[m];
            const double nup = mt->k1[m] * mt->k2[m] * e;
            const double acc = face_geo(g, 0) * (fw[0] * fa[0] + fw[1] * fa[1]) +
                               face_geo(g, 1) * (fw[2] * fa[2] + fw[3] * fa[3]) +
                               face_geo(g, 2) * (fw[4] * fa[4] + fw[5] * fa[5]);
            double *r = cellv + c * kCellRec;
            r[0] = nu;
            r[1] = nup * acc;
            r[2] = B[0];
            r[3] = B[1];
            r[4] = B[2];
            if (m == mat) v[0] = 0.5 * e * acc;
        }
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Edge pass: out[e] = [C^T (M_nu C u + q)]_e for every conducting edge e,
// four lanes per edge (one face each, summed over the lane group).
__global__ void __launch_bounds__(256)
    k_adj_edge(Geo g, const int *__restrict__ cslot, int nc, const double *__restrict__ cellv,
               const double *__restrict__ u, double *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = t >> 2;
    const int q = (int)(t & 3);
    double val = 0.0;
    if (e < nc) {
        const int64_t slot = cslot[e];
        const int c = (int)(slot / g.S);
        int i, j, k;
        decode(g, slot - (int64_t)c * g.S, i, j, k);
        const int c1 = c == 2 ? 0 : c + 1, c2 = c == 0 ? 2 : c - 1;
        // the four faces of the edge: normal, shift, sign
        const int n = q < 2 ? c2 : c1;
        const int sh = q == 1 ? c1 : (q == 3 ? c2 : -1);
        const double sign = (q == 0 || q == 3) ? 1.0 : -1.0;
        int f[3] = {i, j, k};
        if (sh >= 0) f[sh] -= 1;
        int ca[3] = {f[0], f[1], f[2]};
        ca[n] -= 1;
        const int64_t cA = ((int64_t)ca[2] * g.ny + ca[1]) * g.nx + ca[0];
        const int64_t cB = ((int64_t)f[2] * g.ny + f[1]) * g.nx + f[0];
        const double *rA = cellv + cA * kCellRec, *rB = cellv + cB * kCellRec;
        const double mnu = face_geo(g, n) * 0.5 * (rA[0] + rB[0]);
        const double qf = 0.5 * (rA[1] * rA[2 + n] + rB[1] * rB[2 + n]) / face_area(g, n);
        val = sign * (mnu * face_flux(g, u, n, f[0], f[1], f[2]) + qf);
    }
    val += __shfl_xor(val, 1, 64);
    val += __shfl_xor(val, 2, 64);
    if (e < nc && q == 0) out[e] = val;
}

// Adjoint update of one step (compact vectors):
//   d = a_m - a_m1;  mu = (2/dt) M_c (d - d_next) + mu_next - dt jt  (terminal:
//   (2/dt) M_c d), d_next <- d, and the sigma partial
//   (1/dt) d Phi d - mu M_c^{-1} Phi d.
__global__ void __launch_bounds__(256)
    k_adj_mu(int nc, const double *__restrict__ a_m, const double *__restrict__ a_m1,
             const double *mu_next, double *d_next, const double *__restrict__ minv,
             const double *__restrict__ phi, const double *__restrict__ jt, double dt,
             int terminal, double *mu_out, double *part)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (e < nc) {
        const double d = a_m[e] - a_m1[e];
        const double mc = 1.0 / minv[e];
        double mu = (2.0 / dt) * mc * d;
        if (!terminal) mu += -(2.0 / dt) * mc * d_next[e] + mu_next[e] - dt * jt[e];
        mu_out[e] = mu;
        d_next[e] = d;
        v[0] = d * phi[e] * d / dt - mu * minv[e] * phi[e] * d;
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// w = M_c^{-1} mu scattered into the conducting slots of y (y's other slots
// are left as they are)
__global__ void k_adj_w(const int *__restrict__ cslot, int nc, const double *__restrict__ mu,
                        const double *__restrict__ minv, double *y)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nc) y[cslot[e]] = minv[e] * mu[e];
}

// Joule loss partial of one step: (1/dt) (a_new - a_old)^T M_c (a_new - a_old)
__global__ void __launch_bounds__(256)
    k_adj_loss(int nc, const double *__restrict__ a_new, const double *__restrict__ a_old,
               const double *__restrict__ minv, double dt, double *part)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (e < nc) {
        const double d = a_new[e] - a_old[e];
        v[0] = d * d / (minv[e] * dt);
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// acc += coef * sum(part[0..nb))  (one block, fixed order)
__global__ void k_adj_accum(const double *part, int nb, double coef, double *acc)
{
    double s[1];
    reduce_partials<1>(part, nb, 1, s);
    if (threadIdx.x == 0) *acc += coef * s[0];
}

__global__ void k_adj_zero(double *acc, int n)
{
    if ((int)threadIdx.x < n) acc[threadIdx.x] = 0.0;
}

// ------------------------------------------------------------- launchers
static int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per); }

void adj_cell_init(double *cellv, int64_t ncell, double nu0, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_cell_init, dim3(blocks_for(ncell, 256)), dim3(256), 0, st, cellv,
                       ncell, nu0);
}

int adj_cell(const Geo &g, const Mats *mt, const uint8_t *cmat, const double *a, const double *w,
             double *cellv, int mat, const int lo[3], const int hi[3], double *part,
             hipStream_t st)
{
    const int ext[3] = {hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1};
    const int64_t cnt = (int64_t)ext[0] * ext[1] * ext[2];
    const int nb = std::max(1, blocks_for(cnt, 256));
    hipLaunchKernelGGL(k_adj_cell, dim3(nb), dim3(256), 0, st, g, mt, cmat, a, w, cellv, mat,
                       lo[0], lo[1], lo[2], ext[0], ext[1], ext[2], part);
    return nb;
}

void adj_edge(const Geo &g, const int *cslot, int nc, const double *cellv, const double *u,
              double *out, hipStream_t st)
{
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_adj_edge, dim3(blocks_for(4 * (int64_t)nc, 256)), dim3(256), 0, st, g,
                       cslot, nc, cellv, u, out);
}

int adj_mu(int nc, const double *a_m, const double *a_m1, const double *mu_next, double *d_next,
           const double *minv, const double *phi, const double *jt, double dt, int terminal,
           double *mu_out, double *part, hipStream_t st)
{
    const int nb = std::max(1, blocks_for(nc, 256));
    hipLaunchKernelGGL(k_adj_mu, dim3(nb), dim3(256), 0, st, nc, a_m, a_m1, mu_next, d_next,
                       minv, phi, jt, dt, terminal, mu_out, part);
    return nb;
}

void adj_w(const int *cslot, int nc, const double *mu, const double *minv, double *y,
           hipStream_t st)
{
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_adj_w, dim3(blocks_for(nc, 256)), dim3(256), 0, st, cslot, nc, mu, minv,
                       y);
}

int adj_loss(int nc, const double *a_new, const double *a_old, const double *minv, double dt,
             double *part, hipStream_t st)
{
    const int nb = std::max(1, blocks_for(nc, 256));
    hipLaunchKernelGGL(k_adj_loss, dim3(nb), dim3(256), 0, st, nc, a_new, a_old, minv, dt, part);
    return nb;
}

void adj_accum(const double *part, int nb, double coef, double *acc, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_accum, dim3(1), dim3(256), 0, st, part, nb, coef, acc);
}

void adj_zero(double *acc, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_zero, dim3(1), dim3(64), 0, st, acc, n);
}


// ------------------------------------------------- forward Jacobian J_N v
// J_N(a) v = [C^T (M_nu(a) C v + dM_nu(a; v) C a)]_C with, per conducting
// cell, d nu = nu'(s) 2 B . dB (B, dB the cell flux densities of a and v,
// s = |B|^2) and a face's d M_nu the mean of its two cells' d nu times dual
// length over area (the derivative of the face-averaged reluctivity).
// Cell pass over the conductor's bounding box: records nu and d nu.
__global__ void __launch_bounds__(256)
    k_jn_cell(Geo g, const Mats *__restrict__ mt, const uint8_t *__restrict__ cmat,
              const double *__restrict__ a, const double *__restrict__ v, double *cellv, int lo0,
              int lo1, int lo2, int ex, int ey, int ez)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cnt = (int64_t)ex * ey * ez;
    if (t >= cnt) return;
    const int64_t exy = (int64_t)ex * ey;
    const int kk = (int)(t / exy);
    const int64_t rem = t - (int64_t)kk * exy;
    const int jj = (int)(rem / ex), ii = (int)(rem - (int64_t)jj * ex);
    const int i = ii + lo0, j = jj + lo1, k = kk + lo2;
    const int64_t c = ((int64_t)k * g.ny + j) * g.nx + i;
    const int m = cmat[c];
    if (!m) return;
    double B[3], dB[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        int q[3] = {i, j, k};
        const double fa0 = face_flux(g, a, n, q[0], q[1], q[2]);
        const double fv0 = face_flux(g, v, n, q[0], q[1], q[2]);
        q[n] += 1;
        const double fa1 = face_flux(g, a, n, q[0], q[1], q[2]);
        const double fv1 = face_flux(g, v, n, q[0], q[1], q[2]);
        B[n] = 0.5 * (fa0 + fa1) / face_area(g, n);
        dB[n] = 0.5 * (fv0 + fv1) / face_area(g, n);
    }
    const double s = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    const double e = exp(mt->k2[m] * s);
    double *r = cellv + c * kCellRec;
    r[0] = mt->k1[m] * e + mt->k3[m];
    r[1] = mt->k1[m] * mt->k2[m] * e * 2.0 * (B[0] * dB[0] + B[1] * dB[1] + B[2] * dB[2]);
}

// Edge pass: out[e] = sum over the four faces of edge e of
// sign (M_nu C u + dM_nu C a)_f, with u = v on C and -K_n^+ K_cn^T v on N
// this is J_N(a) v - S v on the conducting edges (four lanes per edge).
__global__ void __launch_bounds__(256)
    k_jn_edge(Geo g, const int *__restrict__ cslot, int nc, const double *__restrict__ cellv,
              const double *__restrict__ u, const double *__restrict__ a, double *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e = t >> 2;
    const int q = (int)(t & 3);
    double val = 0.0;
    if (e < nc) {
        const int64_t slot = cslot[e];
        const int c = (int)(slot / g.S);
        int i, j, k;
        decode(g, slot - (int64_t)c * g.S, i, j, k);
        const int c1 = c == 2 ? 0 : c + 1, c2 = c == 0 ? 2 : c - 1;
        const int n = q < 2 ? c2 : c1;
        const int sh = q == 1 ? c1 : (q == 3 ? c2 : -1);
        const double sign = (q == 0 || q == 3) ? 1.0 : -1.0;
        int f[3] = {i, j, k};
        if (sh >= 0) f[sh] -= 1;
        int ca[3] = {f[0], f[1], f[2]};
        ca[n] -= 1;
        const int64_t cA = ((int64_t)ca[2] * g.ny + ca[1]) * g.nx + ca[0];
        const int64_t cB = ((int64_t)f[2] * g.ny + f[1]) * g.nx + f[0];
        const double *rA = cellv + cA * kCellRec, *rB = cellv + cB * kCellRec;
        const double geo = face_geo(g, n);
        const double mnu = geo * 0.5 * (rA[0] + rB[0]);
        const double dm = geo * 0.5 * (rA[1] + rB[1]);
        val = sign * (mnu * face_flux(g, u, n, f[0], f[1], f[2]) +
                      dm * face_flux(g, a, n, f[0], f[1], f[2]));
    }
    val += __shfl_xor(val, 1, 64);
    val += __shfl_xor(val, 2, 64);
    if (e < nc && q == 0) out[e] = val;
}

void jn_cell(const Geo &g, const Mats *mt, const uint8_t *cmat, const double *a, const double *v,
             double *cellv, const int lo[3], const int hi[3], hipStream_t st)
{
    const int ext[3] = {hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1};
    const int64_t cnt = (int64_t)ext[0] * ext[1] * ext[2];
    if (cnt <= 0) return;
    hipLaunchKernelGGL(k_jn_cell, dim3(blocks_for(cnt, 256)), dim3(256), 0, st, g, mt, cmat, a, v,
                       cellv, lo[0], lo[1], lo[2], ext[0], ext[1], ext[2]);
}

void jn_edge(const Geo &g, const int *cslot, int nc, const double *cellv, const double *u,
             const double *a, double *out, hipStream_t st)
{
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_jn_edge, dim3(blocks_for(4 * (int64_t)nc, 256)), dim3(256), 0, st, g,
                       cslot, nc, cellv, u, a, out);
}

// ------------------------------------------------- stability estimate (eq. 8)
// Power method on B = (X^T - S) M_c^{-1}, the transpose of M_c^{-1} (X - S)
// (X = J_N(a) or K_c(nu(a)); same eigenvalues), on compact conducting-edge
// vectors: one block, fixed-order sums (deterministic).

// counter-based start vector: splitmix64 of the edge's list position, uniform
// in [-1/2, 1/2), normalised to unit Euclidean length
__device__ __forceinline__ double unit_hash(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

__global__ void __launch_bounds__(1024) k_power_init(int nc, double *v)
{
    double s[1] = {0.0};
    for (int e = threadIdx.x; e < nc; e += blockDim.x) {
        const double x = unit_hash((uint64_t)e);
        v[e] = x;
        s[0] += x * x;
    }
    block_sum<1>(s);
    const double inv = s[0] > 0.0 ? 1.0 / sqrt(s[0]) : 0.0;
    for (int e = threadIdx.x; e < nc; e += blockDim.x) v[e] *= inv;
}

// y = B v for the unit iterate v: lambda = ||y|| (stored), v <- y / ||y||;
// rec (may be null) receives {lambda, v^T y}
__global__ void __launch_bounds__(1024)
    k_power_norm(int nc, const double *__restrict__ y, double *v, double *lam, double *rec)
{
    double s[2] = {0.0, 0.0};
    for (int e = threadIdx.x; e < nc; e += blockDim.x) {
        const double ye = y[e];
        s[0] += ye * ye;
        s[1] += v[e] * ye;
    }
    block_sum<2>(s);
    const double l = sqrt(s[0]);
    const double inv = l > 0.0 ? 1.0 / l : 0.0;
    for (int e = threadIdx.x; e < nc; e += blockDim.x) v[e] = y[e] * inv;
    if (threadIdx.x == 0) {
        *lam = l;
        if (rec) {
            rec[0] = l;
            rec[1] = s[1];
        }
    }
}

void power_init(int nc, double *v, hipStream_t st)
{
    if (nc > 0) hipLaunchKernelGGL(k_power_init, dim3(1), dim3(1024), 0, st, nc, v);
}

void power_norm(int nc, const double *y, double *v, double *lam, double *rec, hipStream_t st)
{
    if (nc > 0) hipLaunchKernelGGL(k_power_norm, dim3(1), dim3(1024), 0, st, nc, y, v, lam, rec);
}

}  // namespace ec
