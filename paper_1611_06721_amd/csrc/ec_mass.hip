// ec_mass.hip -- the consistent conductivity matrix on gfx950: M_c x, the
// Jacobi-PCG for M_c y = g, and the slot product of an SPE history push of
// that sequence (the last paragraph of Sec. III: a non-diagonal M_c makes
// M_c^{-1} in eq. (6) a further sequence of linear systems).
//
// M_c couples each conducting edge with the parallel edges of the (up to
// four) conducting cells around it: at most nine entries per row, stored as
// ELL columns over the compact conducting-edge list (entry q of row e at
// q * nc + e, so a wave reads consecutive rows).  Vectors are compact.
//
// PCG: the single-reduction Jacobi form of the K_n solves (Chronopoulos and
// Gear; same records, partials and decisions), with u = D^-1 r, w = M u:
//   p_i = u_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}
//   x += alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i,
//   w_{i+1} = M D^-1 r_{i+1}, evaluated from r_i, w_i, s_{i-1} at the row's
//   neighbours in the same kernel (one grid-wide reduction per iteration).
#include "ec_device.h"

namespace ec {

// rows of the block's share (grid-stride)
template <typename F>
__device__ __forceinline__ void for_rows(int nc, F fn)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nc; e += gridDim.x * blockDim.x)
        fn(e);
}

__global__ void __launch_bounds__(256) k_mass_apply(MassOp M, const double *__restrict__ x,
                                                     double *__restrict__ y)
{
    for_rows(M.nc, [&](int e) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < kMassNnz; ++q) {
            const int f = M.idx[(int64_t)q * M.nc + e];
            if (f >= 0) v += M.val[(int64_t)q * M.nc + e] * x[f];
        }
        y[e] = v;
    });
}

void mass_apply(const MassOp &M, const double *x, double *y, hipStream_t st)
{
    if (M.nc <= 0) return;
    hipLaunchKernelGGL(k_mass_apply, dim3(mass_blocks(M.nc)), dim3(256), 0, st, M, x, y);
}

int mass_blocks(int nc) { return std::max(1, std::min((nc + 255) / 256, kMaxBlocks)); }

// Init: r0 = b (zero start, x = 0) or the start vector's residual (rb[0],
// START_DEV with a basis), w0 = M D^-1 r0, partials (gamma0, delta0, |r0|^2,
// |b|^2) into part[0].  Block 0 writes the record.
__global__ void __launch_bounds__(256) k_mass_cg_init(MassCg a)
{
    const MassOp &M = a.M;
    const bool zero = a.mode == START_ZERO || (a.mode == START_DEV && a.seq->zero_start);
    double *r0 = a.rb[0], *w0 = a.wb[0];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for_rows(M.nc, [&](int e) {
        double w = 0.0;
#pragma unroll
        for (int q = 0; q < kMassNnz; ++q) {
            const int f = M.idx[(int64_t)q * M.nc + e];
            if (f >= 0) w += M.val[(int64_t)q * M.nc + e] * (M.dinv[f] * (zero ? a.b[f] : r0[f]));
        }
        const double bv = a.b[e];
        const double rv = zero ? bv : r0[e];
        const double u = M.dinv[e] * rv;
        v[0] += u * rv;
        v[1] += w * u;
        v[2] += rv * rv;
        v[3] += bv * bv;
        w0[e] = w;
    });
    // a second pass: r0 and x of a zero start (their old values were read above)
    if (zero)
        for_rows(M.nc, [&](int e) {
            r0[e] = a.b[e];
            a.x[e] = 0.0;
        });
    block_sum<4>(v);
    if (threadIdx.x == 0) {
        for (int q = 0; q < 4; ++q) a.part[(int64_t)blockIdx.x * 4 + q] = v[q];
        if (blockIdx.x == 0) {
            CgCtl c0{};
            c0.done = 0;
            c0.status = EC_OK;
            a.ctl[0] = c0;
        }
    }
}

__global__ void __launch_bounds__(256) k_mass_cg_iter(MassCg a, int it)
{
    __shared__ CgCtl s_c;
    __shared__ double s_beta;
    if (a.ctl[it & 1].done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl[(it + 1) & 1] = a.ctl[it & 1];
        return;
    }
    double t[4];
    part_load(a.part + (int64_t)(it & 1) * 4 * kMaxBlocks, gridDim.x, t);
    block_sum<4>(t);
    if (threadIdx.x == 0) {
        double beta;
        s_c = cg_state(a.ctl[it & 1], t, it, a.rtol, a.maxit, beta);
        s_beta = beta;
        if (blockIdx.x == 0) {
            CgCtl o = s_c;
            if (!o.done) o.it = it + 1;
            a.ctl[(it + 1) & 1] = o;
        }
    }
    __syncthreads();
    if (s_c.done) return;
    const MassOp &M = a.M;
    const double alpha = s_c.alpha, beta = s_beta;
    const bool first = it == 0;
    const double *rc = a.rb[it & 1], *wc = a.wb[it & 1], *sp = a.sb[(it + 1) & 1];
    double *rn = a.rb[(it + 1) & 1], *wn = a.wb[(it + 1) & 1], *sc = a.sb[it & 1];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for_rows(M.nc, [&](int e) {
        double w1 = 0.0;
#pragma unroll
        for (int q = 0; q < kMassNnz; ++q) {
            const int f = M.idx[(int64_t)q * M.nc + e];
            if (f >= 0) {
                const double tf = first ? M.dinv[f] * (rc[f] - alpha * wc[f])
                                        : M.dinv[f] * (rc[f] - alpha * (wc[f] + beta * sp[f]));
                w1 += M.val[(int64_t)q * M.nc + e] * tf;
            }
        }
        const double d = M.dinv[e];
        const double rv = rc[e], wv = wc[e];
        const double si = first ? wv : wv + beta * sp[e];
        const double pi = first ? d * rv : d * rv + beta * a.p[e];
        a.x[e] += alpha * pi;
        a.p[e] = pi;
        sc[e] = si;
        const double r1 = rv - alpha * si;
        rn[e] = r1;
        wn[e] = w1;
        const double u1 = d * r1;
        v[0] += u1 * r1;
        v[1] += w1 * u1;
        v[2] += r1 * r1;
    });
    block_sum<4>(v);
    if (threadIdx.x == 0) {
        double *Pout = a.part + (int64_t)((it + 1) & 1) * 4 * kMaxBlocks;
        for (int q = 0; q < 4; ++q) Pout[(int64_t)blockIdx.x * 4 + q] = v[q];
    }
}

// final decision after `iters` iteration kernels, the record and counters
__global__ void __launch_bounds__(256) k_mass_cg_fin(MassCg a, int iters)
{
    double t[4];
    reduce_partials<4>(a.part + (int64_t)(iters & 1) * 4 * kMaxBlocks, a.blocks, 4, t);
    if (threadIdx.x != 0) return;
    double beta;
    CgCtl c = cg_state(a.ctl[iters & 1], t, iters, a.rtol, a.maxit + 1, beta);
    int st = c.status;
    if (!c.done) st = EC_ERR_NOT_CONVERGED;
    if (a.seq && c.it == 0 && a.seq->method == EC_SV_SPE) a.seq->push_on = 0;
    if (a.info) {
        const double bb = c.bb;
        a.info->iters = c.it;
        a.info->outer_iters = 0;
        a.info->rel_res = bb > 0.0 ? sqrt(c.rho / bb) : 0.0;
        a.info->b_norm = sqrt(bb);
        a.info->r0_rel = bb > 0.0 ? sqrt(c.rho0 / bb) : 0.0;
        a.info->basis_cols = a.seq ? a.seq->k : 0;
        a.info->pod_info = 1.0;
        a.info->status = (st == EC_OK && a.seq && a.seq->flags) ? EC_ERR_SINGULAR_PROJ : st;
    }
    if (a.ctrl) {
        a.ctrl->mass_solves += 1;
        a.ctrl->mass_iters += c.it;
        if (st < a.ctrl->worst) a.ctrl->worst = st;
    }
}

void mass_cg_init(const MassCg &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_mass_cg_init, dim3(a.blocks), dim3(256), 0, st, a);
}
void mass_cg_iter(const MassCg &a, int it, hipStream_t st)
{
    hipLaunchKernelGGL(k_mass_cg_iter, dim3(a.blocks), dim3(256), 0, st, a, it);
}
void mass_cg_fin(const MassCg &a, int iters, hipStream_t st)
{
    hipLaunchKernelGGL(k_mass_cg_fin, dim3(1), dim3(256), 0, st, a, iters);
}

// Slot product of an SPE push of the mass sequence: ycopy = M x and
// xcopy = x at column *slot (ld apart), ypen = M x (the projected matrix has
// no grad-div term here); every block first runs the acceptance test of the
// push (the dense step OP_SPE_PUSH3 on |x|^2 from the partials pin) and
// leaves unless the column is accepted; block 0 stores the test's results.
__global__ void __launch_bounds__(256)
    k_mass_slots(MassOp M, int64_t ld, const double *__restrict__ x, double *ycopy,
                 double *xcopy, double *ypen, const int *slot, SeqDev *sq, const double *pin,
                 double tol)
{
    __shared__ double s_v[1];
    __shared__ int s_acc;
    reduce_rows<1>(pin, 1, 1, s_v);
    if (threadIdx.x == 0) {
        const int k = sq->k;
        const double rho = sqrt(s_v[0]);
        const int acc = (sq->active && rho > tol * sq->xnorm && k + 1 < kMaxWin) ? 1 : 0;
        if (blockIdx.x == 0) {
            sq->rho = rho;
            sq->accept = acc;
            if (acc) sq->s[k] = 1.0 / rho;
            sq->ncol_md = k + 1;
        }
        s_acc = acc;
    }
    __syncthreads();
    if (!s_acc) return;
    const int64_t col = (int64_t)(*slot) * ld;
    for_rows(M.nc, [&](int e) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < kMassNnz; ++q) {
            const int f = M.idx[(int64_t)q * M.nc + e];
            if (f >= 0) v += M.val[(int64_t)q * M.nc + e] * x[f];
        }
        ycopy[col + e] = v;
        xcopy[col + e] = x[e];
        ypen[e] = v;
    });
}

void mass_slots(const MassOp &M, int64_t ld, const double *x, double *ycopy, double *xcopy,
                double *ypen, const int *slot, SeqDev *sq, const double *pin, double tol,
                hipStream_t st)
{
    hipLaunchKernelGGL(k_mass_slots, dim3(mass_blocks(M.nc)), dim3(256), 0, st, M, ld, x, ycopy,
                       xcopy, ypen, slot, sq, pin, tol);
}

// a_c^m = a_c^{m-1} - dt y on the conducting slots (dt of the step's record)
__global__ void k_mass_axpy(const int *__restrict__ cslot, int nc, const double *__restrict__ A,
                            const double *__restrict__ y, const Ctrl *ctrl, double *out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc) return;
    const int64_t s = cslot[e];
    out[s] = A[s] - ctrl->dt * y[e];
}

void mass_axpy(const int *cslot, int nc, const double *A, const double *y, const Ctrl *ctrl,
               double *out, hipStream_t st)
{
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_mass_axpy, dim3((nc + 255) / 256), dim3(256), 0, st, cslot, nc, A, y,
                       ctrl, out);
}

}  // namespace ec
