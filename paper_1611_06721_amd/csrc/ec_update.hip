// ec_update.hip -- the conducting-region part of the explicit Euler step on
// gfx950, and small state/control kernels.
//
// For every conducting edge e (eq. 6 with the sign of eq. 5a):
//   g_e = [C^T M_nu(a_c) C (a_c (+) y)]_e,  y = s_j - s_c on nonconducting edges,
//   a_c,e <- a_c,e - dt g_e / M_sigma,e.
// The reluctivity of a conducting cell follows the Brauer curve
// nu = k1 exp(k2 |B|^2) + k3 of its flux density B (mean of opposite face
// fluxes); a face's reluctance is the mean of its two cells' nu times dual
// length over area.  Four lanes serve one edge: lane q evaluates the nu of
// cell q around the edge and the contribution of face q, and the four
// contributions are summed with lane shuffles.
#include <math.h>

#include "ec_device.h"

namespace ec {

// state value of edge (c, i, j, k): a_c on conducting, the N operand on
// nonconducting, 0 on Dirichlet edges
struct EdgeVal {
    const Geo &g;
    const UpdArgs &a;
    __device__ double operator()(int c, int i, int j, int k) const
    {
        const int64_t nn = ((int64_t)k * g.py + j) * g.px + i;
        const int64_t ix = (int64_t)c * g.S + nn;
        const int cl = edge_cls(g, c, i, j, k, nn);
        if (cl == 1) return a.A[ix];
        if (cl == 2) return a.xn ? a.xn[ix] : a.sj[ix] - (a.sc ? a.sc[ix] : 0.0);
        return 0.0;
    }
};

// flux through the face with normal n anchored at node p (cyclic axes
// n1 = n+1, n2 = n+2): V(n1, p) + V(n2, p + e_n1) - V(n1, p + e_n2) - V(n2, p)
template <typename F>
__device__ __forceinline__ double face_flux(F V, int n, const int (&p)[3])
{
    const int n1 = (n + 1) % 3, n2 = (n + 2) % 3;
    int q1[3] = {p[0], p[1], p[2]}, q2[3] = {p[0], p[1], p[2]};
    q1[n1] += 1;
    q2[n2] += 1;
    return V(n1, p[0], p[1], p[2]) + V(n2, q1[0], q1[1], q1[2]) - V(n1, q2[0], q2[1], q2[2]) -
           V(n2, p[0], p[1], p[2]);
}

__device__ __forceinline__ void update_body(const UpdArgs &a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int e_idx = t >> 2, q = t & 3;
    if (e_idx >= a.nc) return;                 // whole 4-lane groups leave together
    const Geo &g = a.g;
    const int64_t e = a.cslot[e_idx];
    const int c = (int)(e / g.S);
    int p[3];
    decode(g, e - (int64_t)c * g.S, p[0], p[1], p[2]);
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;   // cyclic axes across the edge
    const double h[3] = {g.hx, g.hy, g.hz};

    // nu of cell q: offsets (q & 1) - 1 along a1 and (q >> 1) - 1 along a2
    int cell[3] = {p[0], p[1], p[2]};
    cell[a1] += (q & 1) - 1;
    cell[a2] += (q >> 1) - 1;
    double nu;
    {
        const int m = a.cmat[((int64_t)cell[2] * g.ny + cell[1]) * g.nx + cell[0]];
        if (m == 0) {
            nu = a.m->nu0;
        } else if (a.m->k1[m] == 0.0) {
            nu = a.m->k3[m];
        } else {
            const double *NS = a.nustate ? a.nustate : a.A;
            auto W = [&](int cc, int ii, int jj, int kk) -> double {
                return NS[(int64_t)cc * g.S + ((int64_t)kk * g.py + jj) * g.px + ii];
            };
            double b2 = 0.0;
            for (int n = 0; n < 3; ++n) {
                int pc[3] = {cell[0], cell[1], cell[2]};
                const double f0 = face_flux(W, n, pc);
                pc[n] += 1;
                const double f1 = face_flux(W, n, pc);
                const double B = 0.5 * (f0 + f1) / (h[(n + 1) % 3] * h[(n + 2) % 3]);
                b2 += B * B;
            }
            nu = a.m->k1[m] * exp(a.m->k2[m] * b2) + a.m->k3[m];
        }
    }
    const double n0 = __shfl(nu, 0, 4), n1v = __shfl(nu, 1, 4), n2v = __shfl(nu, 2, 4),
                 n3 = __shfl(nu, 3, 4);
    // face q: 0: normal a2 at p (+, cells 1,3); 1: normal a2 at p - e_a1 (-, cells 0,2);
    //         2: normal a1 at p (-, cells 2,3); 3: normal a1 at p - e_a2 (+, cells 0,1)
    int fp[3] = {p[0], p[1], p[2]};
    int nrm;
    double sgn, nsum;
    if (q == 0) { nrm = a2; sgn = 1.0; nsum = n1v + n3; }
    else if (q == 1) { nrm = a2; sgn = -1.0; nsum = n0 + n2v; fp[a1] -= 1; }
    else if (q == 2) { nrm = a1; sgn = -1.0; nsum = n2v + n3; }
    else { nrm = a1; sgn = 1.0; nsum = n0 + n1v; fp[a2] -= 1; }
    const EdgeVal V{g, a};
    const double wgeo = h[nrm] / (h[(nrm + 1) % 3] * h[(nrm + 2) % 3]);
    double r = sgn * 0.5 * nsum * wgeo * face_flux(V, nrm, fp);
    r += __shfl_xor(r, 1, 4);
    r += __shfl_xor(r, 2, 4);
    if (q == 0) {
        if (a.gout) {
            a.gout[e_idx] = r;
        } else if (a.apply) {
            a.out[e] = r;
        } else {
            const double dt = a.ctrl ? a.ctrl->dt : a.dt;
            a.out[e] = a.A[e] - dt * r * a.minv[e_idx];
        }
    }
}

__global__ void __launch_bounds__(256) k_update(UpdArgs a)
{
    update_body(a);
}

// one instance of a batch per block row (the grid covers the largest n_c)
__global__ void __launch_bounds__(256) k_update_tab(const UpdArgs *tab)
{
    update_body(tab[blockIdx.y]);
}

void update_c(const UpdArgs &a, hipStream_t st)
{
    if (a.nc <= 0) return;
    const int64_t threads = 4 * (int64_t)a.nc;
    hipLaunchKernelGGL(k_update, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, a);
}

void update_c_tab(const UpdArgs *tab, int n, int nc_max, hipStream_t st)
{
    if (nc_max <= 0) return;
    const int64_t threads = 4 * (int64_t)nc_max;
    hipLaunchKernelGGL(k_update_tab, dim3((unsigned)((threads + 255) / 256), n), dim3(256), 0, st,
                       tab);
}

// -------------------------------------------------- state and step control
// A = a_c (+) (s_j - s_c): a_c on conducting edges of ac, the solutions on
// nonconducting edges (both zero elsewhere), eq. (7).
__global__ void k_finish(int64_t n, double *A, const double *ac, const double *sj,
                         const double *sc, Ctrl *ctrl, int bump)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        A[e] = ac[e] + (sj[e] - sc[e]);
    if (bump && blockIdx.x == 0 && threadIdx.x == 0) ctrl->n_steps += 1;
}

void finish_state(const Geo &g, double *A, const double *ac, const double *sj, const double *sc,
                  Ctrl *ctrl, int bump, hipStream_t st)
{
    const int blocks = (int)std::min<int64_t>((g.npad + 255) / 256, 2048);
    hipLaunchKernelGGL(k_finish, dim3(blocks), dim3(256), 0, st, g.npad, A, ac, sj, sc, ctrl, bump);
}

// one instance of a batch per block row (grid-stride over its own length)
__global__ void k_finish_tab(const FinArgs *tab)
{
    const FinArgs &f = tab[blockIdx.y];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < f.n; e += stride)
        f.A[e] = f.ac[e] + (f.sj[e] - f.sc[e]);
    if (blockIdx.x == 0 && threadIdx.x == 0) f.ctrl->n_steps += 1;
}

void finish_state_tab(const FinArgs *tab, int n, int64_t npad_max, hipStream_t st)
{
    const int blocks = (int)std::min<int64_t>((npad_max + 255) / 256, 2048);
    hipLaunchKernelGGL(k_finish_tab, dim3(blocks, n), dim3(256), 0, st, tab);
}

// i_S(t_m) of the source waveforms (DC, sine, linear ramp, 1 - exp(-t/tau)).
__device__ __forceinline__ void step_begin_body(Ctrl *ctrl, int64_t m_arg, int wf, double amp,
                                                double freq, double tau, int64_t ramp, double dt,
                                                const double *lam, double safety)
{
    const int64_t m = m_arg >= 0 ? m_arg : ctrl->step + 1;
    ctrl->step = m;
    double t;
    if (lam) {
        // adaptive step: halve dt until dt lambda <= 2 safety (eq. 8 with a
        // margin); a non-positive or non-finite estimate leaves dt as given
        const double l = *lam;
        double dm = dt;
        if (l > 0.0 && l < 1e300)
            for (int q = 0; q < 64 && dm * l > 2.0 * safety; ++q) dm *= 0.5;
        ctrl->dt = dm;
        t = ctrl->t + dm;
    } else {
        ctrl->dt = dt;
        t = (double)m * dt;
    }
    ctrl->t = t;
    double s = 0.0;
    switch (wf) {
    case EC_WF_DC: s = amp; break;
    case EC_WF_SIN: s = amp * sin(2.0 * M_PI * freq * t); break;
    case EC_WF_RAMP: s = amp * (m >= ramp ? 1.0 : (double)m / (double)ramp); break;
    case EC_WF_EXP: s = amp * (1.0 - exp(-t / tau)); break;
    default: s = 0.0;
    }
    ctrl->scale = s;
}

__global__ void k_step_begin(Ctrl *ctrl, int64_t m_arg, int wf, double amp, double freq,
                             double tau, int64_t ramp, double dt, const double *lam,
                             double safety)
{
    step_begin_body(ctrl, m_arg, wf, amp, freq, tau, ramp, dt, lam, safety);
}

// one instance of a batch per block row
__global__ void k_step_begin_tab(const StepArgs *tab, int64_t m_arg)
{
    const StepArgs &s = tab[blockIdx.y];
    step_begin_body(s.ctrl, m_arg, s.wf, s.amp, s.freq, s.tau, s.ramp, s.dt, s.lam, s.safety);
}

void step_begin_tab(const StepArgs *tab, int n, int64_t m, hipStream_t st)
{
    hipLaunchKernelGGL(k_step_begin_tab, dim3(1, n), dim3(1), 0, st, tab, m);
}

void step_begin(Ctrl *ctrl, int64_t m, int wf, double amp, double freq, double tau, int64_t ramp,
                double dt, hipStream_t st, const double *lam, double safety)
{
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(1), 0, st, ctrl, m, wf, amp, freq, tau, ramp,
                       dt, lam, safety);
}

// A kernel with a 128-byte private segment per lane (more than any other
// kernel of the library needs) that touches no global memory: its volatile
// array lives in scratch, and the value it reads back is never -1.
__global__ void k_scratch_warm(int *never)
{
    volatile int buf[32];
    const int t = (int)threadIdx.x;
    for (int i = 0; i < 32; ++i) buf[i] = t + i;
    const int v = buf[(t * 7) & 31];
    if (v == -1) never[0] = v;
}

void scratch_warm(hipStream_t st)
{
    hipLaunchKernelGGL(k_scratch_warm, dim3(256), dim3(256), 0, st, nullptr);
}

__global__ void k_fill(double *y, double v, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) y[e] = v;
}

void fill(double *y, double v, int64_t n, hipStream_t st)
{
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
    if (blocks > 0) hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, st, y, v, n);
}

__global__ void k_copy_c(const int *cslot, int nc, const double *src, double *dst)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nc) dst[cslot[t]] = src[cslot[t]];
}

void copy_c(const int *cslot, int nc, const double *src, double *dst, hipStream_t st)
{
    if (nc > 0)
        hipLaunchKernelGGL(k_copy_c, dim3((nc + 255) / 256), dim3(256), 0, st, cslot, nc, src, dst);
}

// y = x on edges of class `keep`, 0 elsewhere
__global__ void k_mask_copy(Geo g, const double *x, double *y, int keep)
{
    const int64_t n = g.S;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        int i, j, k;
        decode(g, e, i, j, k);
        for (int c = 0; c < 3; ++c) {
            const int64_t ix = (int64_t)c * g.S + e;
            y[ix] = edge_cls(g, c, i, j, k, e) == keep ? x[ix] : 0.0;
        }
    }
}

void mask_copy(const Geo &g, const double *x, double *y, int keep, hipStream_t st)
{
    const int blocks = (int)std::min<int64_t>((g.S + 255) / 256, 2048);
    hipLaunchKernelGGL(k_mask_copy, dim3(blocks), dim3(256), 0, st, g, x, y, keep);
}

__global__ void k_gather_c(const int *cslot, int nc, const double *src, double *dst)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nc) dst[t] = src[cslot[t]];
}
__global__ void k_scatter_c(const int *cslot, int nc, const double *src, double *dst)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nc) dst[cslot[t]] = src[t];
}
void gather_c(const int *cslot, int nc, const double *src, double *dst, hipStream_t st)
{
    if (nc > 0)
        hipLaunchKernelGGL(k_gather_c, dim3((nc + 255) / 256), dim3(256), 0, st, cslot, nc, src, dst);
}
void scatter_c(const int *cslot, int nc, const double *src, double *dst, hipStream_t st)
{
    if (nc > 0)
        hipLaunchKernelGGL(k_scatter_c, dim3((nc + 255) / 256), dim3(256), 0, st, cslot, nc, src,
                           dst);
}

__global__ void k_negate(const double *x, double *y, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) y[e] = -x[e];
}

void negate(const double *x, double *y, int64_t n, hipStream_t st)
{
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
    if (blocks > 0) hipLaunchKernelGGL(k_negate, dim3(blocks), dim3(256), 0, st, x, y, n);
}

}  // namespace ec
