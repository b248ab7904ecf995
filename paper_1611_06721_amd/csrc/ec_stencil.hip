// ec_stencil.hip -- curl-curl products and the Jacobi-PCG for the
// pseudo-inverse K_n^+ b of eq. (9) on gfx950.
//
// SpMV: y = [K_air x]_N, matrix free (K_n x for x on nonconducting edges,
// K_cn^T x for x on conducting edges; eq. 3 blocks), one thread per node.
//
// PCG (Sec. III; weak gauging of Sec. II): the single-reduction form of
// Jacobi-preconditioned CG (Chronopoulos and Gear), algebraically the same
// iterates as standard PCG.  With u = D^-1 r, w = K_n u:
//   p_i = u_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}     (s = K_n p)
//   x += alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i,  w_{i+1} = K_n D^-1 r_{i+1}
//   gamma = r^T u, delta = w^T u:  beta_{i+1} = gamma_{i+1}/gamma_i,
//   alpha_{i+1} = gamma_{i+1} / (delta_{i+1} - beta_{i+1} gamma_{i+1}/alpha_i)
// One kernel per iteration computes r_{i+1} at the 24 stencil points on the
// fly, so the iteration needs a single grid-wide reduction.  Each kernel
// starts by reducing the previous kernel's block partials (every block, same
// order: no atomics or cache flushes) and derives alpha, beta and the stop
// decision.  Stop: ||r|| <= rtol ||b|| (recursive residual).
#include <math.h>

#include <algorithm>

#include "ec_device.h"

namespace ec {

// ------------------------------------------------------- grad-div penalty
// G^T x at node (i,j,k) when the node is free (interior, and no conducting
// edge ends there), else 0.  G phi puts phi(head) - phi(tail) on an edge.
__device__ __forceinline__ double free_div(const Geo &g, const double *__restrict__ x, int i,
                                           int j, int k)
{
    if (i <= 0 || i >= g.nx || j <= 0 || j >= g.ny || k <= 0 || k >= g.nz) return 0.0;
    const int64_t oj = g.px, ok = (int64_t)g.px * g.py;
    const int64_t n = k * ok + j * oj + i;
    if (edge_cls(g, 0, i, j, k, n) == 1 || edge_cls(g, 0, i - 1, j, k, n - 1) == 1 ||
        edge_cls(g, 1, i, j, k, n) == 1 || edge_cls(g, 1, i, j - 1, k, n - oj) == 1 ||
        edge_cls(g, 2, i, j, k, n) == 1 || edge_cls(g, 2, i, j, k - 1, n - ok) == 1)
        return 0.0;
    const int64_t S = g.S;
    return (x[n - 1] - x[n]) + (x[S + n - oj] - x[S + n]) + (x[2 * S + n - ok] - x[2 * S + n]);
}

// ------------------------------------------------------------- SpMV kernel
// One argument set: y (if given) = K_n x; ycopy/xcopy (if given) receive K_n x
// and x at column *slot (ld apart); ypen (if given, FP64) = K_n x + eta D^T D x
// on nonconducting edges (K_n x for eta = 0); nothing when *active == 0.
template <typename T>
struct SpmvArgs {
    const T *x;
    T *y, *ycopy, *xcopy, *ypen;
    const int *slot, *active;
    double eta;
    SeqDev *pre_seq;         // see SlotArgs
    const double *pin;
    double tol;
};

// Blocks are mapped XCD-contiguously (block b runs on XCD b % 8): each XCD
// sweeps one slab, so the k +- 1 planes of the stencil stay in its own L2.
template <typename T>
__device__ __forceinline__ void spmv_box(const Geo &g, int lo0, int lo1, int lo2, int ex, int ey,
                                         int ez, int tiles, int tpx, int64_t ld,
                                         const SpmvArgs<T> &a)
{
    if constexpr (std::is_same<T, double>::value) {
        if (a.pre_seq) {
            // acceptance test of the pushed column (the dense step of an SPE
            // push): x2 is not numerically in span(q)
            __shared__ double s_v[1];
            __shared__ int s_acc;
            reduce_rows<1>(a.pin, 1, 1, s_v);
            if (threadIdx.x == 0) {
                SeqDev *sq = a.pre_seq;
                const int k = sq->k;
                const double rho = sqrt(s_v[0]);
                const int acc = (sq->active && rho > a.tol * sq->xnorm && k + 1 < kMaxWin) ? 1 : 0;
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
        }
    }
    if (a.active && !*a.active) return;
    const int b = blockIdx.x, tile = (b & 7) * tpx + (b >> 3);
    if (tile >= tiles) return;
    const int64_t t = (int64_t)tile * kTile + threadIdx.x;
    const int64_t cnt = (int64_t)ex * ey * ez;
    if (t >= cnt) return;
    const T *__restrict__ x = a.x;
    T *__restrict__ y = a.y;
    T *__restrict__ ycopy = a.ycopy;
    T *__restrict__ xcopy = a.xcopy;
    T *__restrict__ ypen = a.ypen;
    const double eta = a.eta;
    if (a.slot) {
        if (ycopy) ycopy += (int64_t)(*a.slot) * ld;
        if (xcopy) xcopy += (int64_t)(*a.slot) * ld;
    }
    const int64_t exy = (int64_t)ex * ey;
    const int kk = (int)((double)t * (1.0 / (double)exy) + 1e-7);
    const int64_t rem = t - (int64_t)kk * exy;
    const int jj = (int)((double)rem * (1.0 / (double)ex) + 1e-7);
    const int ii = (int)(rem - (int64_t)jj * ex);
    const int i = ii + lo0, j = jj + lo1, k = kk + lo2;
    const int64_t n = ((int64_t)k * g.py + j) * g.px + i;
    T q[3];
    curlcurl_node<T>(g, n, [&](int, int64_t ia) { return x[ia]; }, q[0], q[1], q[2]);
    double d0 = 0.0, dh[3] = {0.0, 0.0, 0.0};
    if constexpr (std::is_same<T, double>::value) {
        if (ypen && eta > 0.0) {
            d0 = free_div(g, x, i, j, k);
            dh[0] = free_div(g, x, i + 1, j, k);
            dh[1] = free_div(g, x, i, j + 1, k);
            dh[2] = free_div(g, x, i, j, k + 1);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t ix = (int64_t)c * g.S + n;
        const bool nc = edge_cls(g, c, i, j, k, n) == 2;
        const T v = nc ? q[c] : (T)0;
        if (y) y[ix] = v;
        if (ycopy) ycopy[ix] = v;
        if (xcopy) xcopy[ix] = x[ix];
        if constexpr (std::is_same<T, double>::value) {
            if (ypen) {
                double vp = v;
                if (nc && eta > 0.0) vp += eta * (dh[c] - d0);
                ypen[ix] = vp;
            }
        }
    }
}

// Block row blockIdx.y serves argument set a0 or a1 over the same box.
template <typename T>
__global__ void __launch_bounds__(256)
    k_spmv(Geo g, int lo0, int lo1, int lo2, int ex, int ey, int ez, int tiles, int tpx,
           int64_t ld, SpmvArgs<T> a0, SpmvArgs<T> a1)
{
    const SpmvArgs<T> &a = blockIdx.y ? a1 : a0;
    spmv_box<T>(g, lo0, lo1, lo2, ex, ey, ez, tiles, tpx, ld, a);
}

// Block row blockIdx.y serves instance y of a batch over its full box, with
// the block-to-tile map of its own launch (blocks past its grid leave).
__global__ void __launch_bounds__(256) k_spmv_slot_tab(const SlotTab *tab)
{
    const SlotTab &e = tab[blockIdx.y];
    const Geo g = e.g;
    const int ex = g.nx + 1, ey = g.ny + 1, ez = g.nz + 1;
    const int64_t cnt = (int64_t)ex * ey * ez;
    const int tiles = (int)((cnt + kTile - 1) / kTile), tpx = (tiles + 7) / 8;
    if ((int)(blockIdx.x >> 3) >= tpx) return;
    SpmvArgs<double> a{};
    a.x = e.s.x; a.y = e.s.y; a.ycopy = e.s.ycopy; a.xcopy = e.s.xcopy; a.ypen = e.s.ypen;
    a.slot = e.s.slot; a.active = e.s.active; a.eta = e.s.eta;
    a.pre_seq = e.s.pre_seq; a.pin = e.s.pin; a.tol = e.s.tol;
    spmv_box<double>(g, 0, 0, 0, ex, ey, ez, tiles, tpx, e.ld, a);
}

// y = K_n x over each instance's own box (block row per instance)
__global__ void __launch_bounds__(256) k_spmv_box_tab(const BoxTab *tab)
{
    const BoxTab &e = tab[blockIdx.y];
    const int64_t cnt = (int64_t)e.ext[0] * e.ext[1] * e.ext[2];
    if (cnt <= 0) return;
    const int tiles = (int)((cnt + kTile - 1) / kTile), tpx = (tiles + 7) / 8;
    if ((int)(blockIdx.x >> 3) >= tpx) return;
    SpmvArgs<double> a{};
    a.x = e.x;
    a.y = e.y;
    spmv_box<double>(e.g, e.lo[0], e.lo[1], e.lo[2], e.ext[0], e.ext[1], e.ext[2], tiles, tpx, 0,
                     a);
}

int spmv_box_tpx(const int ext[3])
{
    const int64_t cnt = (int64_t)ext[0] * ext[1] * ext[2];
    if (cnt <= 0) return 0;
    const int tiles = (int)((cnt + kTile - 1) / kTile);
    return (tiles + 7) / 8;
}

void spmv_box_tab(const BoxTab *tab, int n, int tpx_max, hipStream_t st)
{
    if (tpx_max <= 0) return;
    hipLaunchKernelGGL(k_spmv_box_tab, dim3(8 * tpx_max, n), dim3(kTile), 0, st, tab);
}

int spmv_slot_tpx(const Geo &g)
{
    const int64_t cnt = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    const int tiles = (int)((cnt + kTile - 1) / kTile);
    return (tiles + 7) / 8;
}

void spmv_slots_tab(const SlotTab *tab, int n, int tpx_max, hipStream_t st)
{
    hipLaunchKernelGGL(k_spmv_slot_tab, dim3(8 * tpx_max, n), dim3(kTile), 0, st, tab);
}

template <typename T>
static void spmv_launch_box(const Geo &g, const int lo[3], const int ext[3], int64_t ld,
                            const SpmvArgs<T> &a0, const SpmvArgs<T> *a1, hipStream_t st)
{
    const int64_t cnt = (int64_t)ext[0] * ext[1] * ext[2];
    if (cnt <= 0) return;
    const int tiles = (int)((cnt + kTile - 1) / kTile);
    const int tpx = (tiles + 7) / 8;
    hipLaunchKernelGGL(k_spmv<T>, dim3(8 * tpx, a1 ? 2 : 1), dim3(kTile), 0, st, g, lo[0], lo[1],
                       lo[2], ext[0], ext[1], ext[2], tiles, tpx, ld, a0, a1 ? *a1 : a0);
}

void spmv(const Geo &g, const double *x, double *y, const int lo[3], const int hi[3],
          hipStream_t st)
{
    const int ext[3] = {hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1};
    SpmvArgs<double> a{};
    a.x = x;
    a.y = y;
    spmv_launch_box<double>(g, lo, ext, 0, a, nullptr, st);
}

static SpmvArgs<double> slot_args(const SlotArgs &s)
{
    SpmvArgs<double> a{};
    a.x = s.x; a.y = s.y; a.ycopy = s.ycopy; a.xcopy = s.xcopy; a.ypen = s.ypen;
    a.slot = s.slot; a.active = s.active; a.eta = s.eta;
    a.pre_seq = s.pre_seq; a.pin = s.pin; a.tol = s.tol;
    return a;
}

void spmv_slots(const Geo &g, int64_t ld, const SlotArgs &s, hipStream_t st, const SlotArgs *s1)
{
    const int lo[3] = {0, 0, 0}, ext[3] = {g.nx + 1, g.ny + 1, g.nz + 1};
    const SpmvArgs<double> a0 = slot_args(s);
    if (s1) {
        const SpmvArgs<double> a1 = slot_args(*s1);
        spmv_launch_box<double>(g, lo, ext, ld, a0, &a1, st);
    } else {
        spmv_launch_box<double>(g, lo, ext, ld, a0, nullptr, st);
    }
}

void spmv_f(const Geo &g, const float *x, float *y, hipStream_t st)
{
    const int lo[3] = {0, 0, 0}, ext[3] = {g.nx + 1, g.ny + 1, g.nz + 1};
    SpmvArgs<float> a{};
    a.x = x;
    a.y = y;
    spmv_launch_box<float>(g, lo, ext, 0, a, nullptr, st);
}

// ------------------------------------------------------------------- CG
__device__ __forceinline__ double dsel(const double (&d)[3], int c)
{
    return c == 0 ? d[0] : (c == 1 ? d[1] : d[2]);
}

// Reduce the [blocks][4] partials of the previous kernel (every block, same
// fixed order: every block obtains bitwise the same sums).
__device__ __forceinline__ void sum_part(const double *P, int nb, double (&t)[4])
{
    reduce_partials<4>(P, nb, 4, t);
}

// Init, phase START_X: r0 = s b - K_n x0, partials (|r0|^2, |b|^2) into part[1].
// Init, phases ZERO / R / R2 / DEV: w0 = K_n D^-1 r0 and partials
// (gamma0 = r0^T D^-1 r0, delta0 = w0^T D^-1 r0, |r0|^2, |b|^2) into part[0].
// Block bid of nb of the init in mode `mode`.
template <typename T>
__device__ __forceinline__ void cg_init_body(const CgArgs<T> &a, int mode, int bid, int nb)
{
    const Geo &g = a.g;
    const int64_t S = g.S;
    const double dd[3] = {g.dinv[0], g.dinv[1], g.dinv[2]};
    const double bs = a.bscale ? *a.bscale : 1.0;
    if (mode == START_DEV) mode = a.seq->zero_start ? START_ZERO : START_R;
    if (mode == START_R && a.start_part) {
        // the start combination's own sums of r0^2 and b^2: a start vector
        // that already meets the tolerance (the test of the first
        // iteration's decision) ends the solve here, with no stencil pass;
        // the iteration kernels then find the record finished
        __shared__ double s_v[3];
        reduce_rows<3>(a.start_part, 3, 3, s_v);
        const double rr = s_v[1], bb = s_v[2];
        const double rtol = a.rtol_dev ? *a.rtol_dev : a.rtol;
        const double tol2 = rtol * rtol * bb;
        if (rr == rr && rr <= 1e300 && (bb == 0.0 || rr <= tol2)) {
            if (bid == 0 && threadIdx.x == 0) {
                CgCtl c0{};
                c0.done = 1;
                c0.status = EC_OK;
                c0.bb = bb;
                c0.tol2 = tol2;
                c0.rho0 = rr;
                c0.rho = rr;
                c0.it = 0;
                a.ctl[0] = c0;
            }
            if (bid == 0 && a.bar)
                for (int q = threadIdx.x; q < kBarWords; q += blockDim.x)
                    a.bar[(int64_t)q * kBarStride] = 0u;
            return;
        }
    }
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    T *r0 = a.rb[0];
    double *P0 = a.part, *P1 = a.part + 4 * (int64_t)kMaxBlocks;
    if (mode == START_X) {
        for_tiles_b(a.tiles, S, bid, nb, [&](int64_t n) {
            int i, j, k;
            decode(g, n, i, j, k);
            T q[3];
            curlcurl_node<T>(g, n, [&](int, int64_t ix) { return a.x[ix]; }, q[0], q[1], q[2]);
            for (int c = 0; c < 3; ++c) {
                const int64_t ix = c * S + n;
                const double kx = edge_cls(g, c, i, j, k, n) == 2 ? (double)q[c] : 0.0;
                const double bv = bs * (double)a.b[ix];
                const T rv = (T)(bv - kx);
                r0[ix] = rv;
                v[0] += (double)rv * (double)rv;
                v[1] += bv * bv;
            }
        });
        block_sum<4>(v);
        if (threadIdx.x == 0)
            for (int q = 0; q < 4; ++q) P1[(int64_t)bid * 4 + q] = v[q];
        return;
    }
    bool zero_all = false;
    if (mode == START_R2) {
        double t[4];
        sum_part(P1, nb, t);
        zero_all = t[1] == 0.0;   // b = 0: the pseudo-inverse solution is x = 0
    }
    for_tiles_b(a.tiles, S, bid, nb, [&](int64_t n) {
        int i, j, k;
        decode(g, n, i, j, k);
        T w[3] = {(T)0, (T)0, (T)0};
        if (zero_all) {
            for (int c = 0; c < 3; ++c) {
                a.x[c * S + n] = (T)0;
                r0[c * S + n] = (T)0;
                a.wb[0][c * S + n] = (T)0;
            }
            return;
        }
        if (mode == START_ZERO) {
            const T tbs = (T)bs;
            curlcurl_node<T>(
                g, n, [&](int c, int64_t ix) { return (T)dsel(dd, c) * (tbs * a.b[ix]); }, w[0],
                w[1], w[2]);
        } else {
            curlcurl_node<T>(g, n, [&](int c, int64_t ix) { return (T)dsel(dd, c) * r0[ix]; },
                             w[0], w[1], w[2]);
        }
        for (int c = 0; c < 3; ++c) {
            const int64_t ix = c * S + n;
            if (edge_cls(g, c, i, j, k, n) != 2) w[c] = (T)0;
            const double bv = bs * (double)a.b[ix];
            double rv;
            if (mode == START_ZERO) {
                r0[ix] = (T)bv;
                a.x[ix] = (T)0;
                rv = (double)(T)bv;
            } else {
                rv = (double)r0[ix];
            }
            a.wb[0][ix] = w[c];
            const double u = dd[c] * rv;
            v[0] += u * rv;
            v[1] += (double)w[c] * u;
            v[2] += rv * rv;
            v[3] += bv * bv;
        }
    });
    block_sum<4>(v);
    if (threadIdx.x == 0) {
        for (int q = 0; q < 4; ++q) P0[(int64_t)bid * 4 + q] = v[q];
        if (bid == 0) {
            CgCtl c0{};
            c0.done = 0;
            c0.status = EC_OK;
            c0.zero_x = zero_all;
            a.ctl[0] = c0;
        }
    }
    // arrival and release words of the tail kernel's barrier
    if (bid == 0 && a.bar)
        for (int q = threadIdx.x; q < kBarWords; q += blockDim.x) a.bar[(int64_t)q * kBarStride] = 0u;
}

template <typename T>
__global__ void __launch_bounds__(256) k_cg_init(CgArgs<T> a)
{
    if (a.skip && *a.skip) return;
    cg_init_body<T>(a, a.mode, blockIdx.x, gridDim.x);
}

// The init of every solve of a batch in one launch (block map as in
// k_cg_iter_batch), all in mode `mode`.
__global__ void __launch_bounds__(256)
    k_cg_init_batch(const CgArgs<double> *__restrict__ tab, const int *__restrict__ inst,
                    const int *__restrict__ off, int mode)
{
    const int i = inst[blockIdx.x];
    const CgArgs<double> &a = tab[i];
    cg_init_body<double>(a, mode, blockIdx.x - off[i], a.blocks);
}

// Block-reduce the thread shares t, decide the state entering iteration it;
// block bid 0 passes the record on.  True (uniformly) when the solve is
// finished.
template <typename T>
__device__ __forceinline__ bool cg_decide(const CgArgs<T> &a, int it, double (&t)[4], CgCtl &s_c,
                                          double &s_beta, int bid)
{
    block_sum<4>(t);
    if (threadIdx.x == 0) {
        double beta;
        const double rtol = (it == 0 && a.rtol_dev) ? *a.rtol_dev : a.rtol;
        s_c = cg_state(a.ctl[it & 1], t, it, rtol, a.maxit, beta);
        s_beta = beta;
        if (bid == 0) {
            CgCtl o = s_c;
            if (!o.done) o.it = it + 1;   // iterations completed after this one
            a.ctl[(it + 1) & 1] = o;
        }
    }
    __syncthreads();
    return s_c.done != 0;
}

template <typename T>
__device__ __forceinline__ void cg_update(const CgArgs<T> &a, int it, const CgCtl &s_c,
                                          double s_beta, int bid, int nb);

// One PCG iteration `it` by the whole grid: reduce the nprev partials of the
// previous iteration (every block, same order), decide, then update x, p, s,
// r, w and leave this iteration's partials.  Returns true (uniformly in every
// block) when the solve was already finished and nothing was updated.
template <typename T>
__device__ __forceinline__ bool cg_iteration(const CgArgs<T> &a, int it, int nprev, CgCtl &s_c,
                                             double &s_beta, int bid, int nb)
{
    double t[4];
    part_load(a.part + (int64_t)(it & 1) * 4 * kMaxBlocks, nprev, t);
    if (cg_decide<T>(a, it, t, s_c, s_beta, bid)) return true;
    cg_update<T>(a, it, s_c, s_beta, bid, nb);
    return false;
}

// The update of iteration it after the decision: x, p, s, r, w of the
// block's tiles and this iteration's partials.
template <typename T>
__device__ __forceinline__ void cg_update(const CgArgs<T> &a, int it, const CgCtl &s_c,
                                          double s_beta, int bid, int nb)
{
    double *Pout = a.part + (int64_t)((it + 1) & 1) * 4 * kMaxBlocks;
    const Geo &g = a.g;
    const int64_t S = g.S;
    const double dd[3] = {g.dinv[0], g.dinv[1], g.dinv[2]};
    const double alpha = s_c.alpha, beta = s_beta;
    const T ta = (T)alpha, tb = (T)beta;
    const T *rc = a.rb[it & 1], *wc = a.wb[it & 1], *sp = a.sb[(it + 1) & 1];
    T *rn = a.rb[(it + 1) & 1], *wn = a.wb[(it + 1) & 1], *sc = a.sb[it & 1];
    const bool first = it == 0;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for_tiles_b(a.tiles, S, bid, nb, [&](int64_t n) {
        int i, j, k;
        decode(g, n, i, j, k);
        T w[3];
        if (first) {
            curlcurl_node<T>(
                g, n, [&](int c, int64_t ix) { return (T)dsel(dd, c) * (rc[ix] - ta * wc[ix]); },
                w[0], w[1], w[2]);
        } else {
            curlcurl_node<T>(
                g, n,
                [&](int c, int64_t ix) {
                    return (T)dsel(dd, c) * (rc[ix] - ta * (wc[ix] + tb * sp[ix]));
                },
                w[0], w[1], w[2]);
        }
        for (int c = 0; c < 3; ++c) {
            const int64_t ix = c * S + n;
            const T d = (T)dsel(dd, c);
            const T rv = rc[ix], wv = wc[ix];
            const T si = first ? wv : wv + tb * sp[ix];
            const T pi = first ? d * rv : d * rv + tb * a.p[ix];
            a.x[ix] += ta * pi;
            a.p[ix] = pi;
            sc[ix] = si;
            const T r1 = rv - ta * si;
            rn[ix] = r1;
            const T w1 = edge_cls(g, c, i, j, k, n) == 2 ? w[c] : (T)0;
            wn[ix] = w1;
            const double u1 = (double)d * (double)r1;
            v[0] += u1 * (double)r1;
            v[1] += (double)w1 * u1;
            v[2] += (double)r1 * (double)r1;
        }
    });
    block_sum<4>(v);
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) Pout[(int64_t)bid * 4 + q] = v[q];
}

// Raw buffer view of a vector of `count` elements for the hoisted iteration:
// a load at element index e reads element e when 0 <= e < count and returns
// 0 otherwise without touching memory (the range check of buffer loads: a
// negative index wraps to an unsigned byte offset beyond the buffer).  Byte
// offsets are 32-bit: count * sizeof(T) < 2^31 (checked where the hoisted
// form is chosen).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_view(const void *p, int64_t bytes)
{
    // dword 3 of a raw (untyped) buffer resource on gfx9-family targets
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}

// the hoisted form runs only with one tile per block, so on at most
// kMaxBlocks tiles: its vectors stay far below 2^31 bytes
static_assert((int64_t)kMaxBlocks * kTile * 3 * 8 < (1ll << 31), "buffer offsets are 32-bit");

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int e)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, e * 4, 0, 0));
}

// The iteration with the node's stencil inputs loaded before the decision,
// for launches where every block sweeps at most one tile: r, w, s at the 24
// stencil positions and the node's own p, x are in flight while the block
// reduces the previous partials, then t = D^-1 (r - alpha (w + beta s)), the
// curl-curl and the update use exactly the expressions of cg_update.  The
// loads go through range-checked buffer views: a stencil position outside
// the vectors (only ever feeding Dirichlet/padding outputs) reads 0, one
// 32-bit index per position instead of a clamped 64-bit address per load.
// This lane's share of the nb block partials of iteration it when one wave
// reduces all of them: records lane, lane + 64, ..., eight in flight per
// lane before any is summed.
__device__ __forceinline__ void part_load_wave(const double *P, int nb, double (&t)[4])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = 0.0;
    for (int b0 = lane; b0 < nb; b0 += 8 * 64) {
        double v[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + u * 64;
            if (b < nb) {
                const double2 *p2 = reinterpret_cast<const double2 *>(P + (int64_t)b * 4);
                const double2 lo = p2[0], hi = p2[1];
                v[u][0] = lo.x; v[u][1] = lo.y; v[u][2] = hi.x; v[u][3] = hi.y;
            } else {
                v[u][0] = v[u][1] = v[u][2] = v[u][3] = 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) t[q] += v[u][q];
    }
}

// Store written through to device-coherent memory (an agent-scope relaxed
// store: the line does not stay dirty in the XCD's L2, so the write-back at
// the end of the kernel has none of these vectors left to flush; 48^3:
// 10.5 instead of 11.0 us per iteration).
template <typename T>
__device__ __forceinline__ void store_wt(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

static_assert(kTile == 256, "the hoisted iteration reduces over four waves");

template <typename T, bool FIRST>
__device__ __forceinline__ bool cg_iter_hoisted_t(const CgArgs<T> &a, int it, int nprev,
                                                  CgCtl &s_c, double &s_beta, int bid)
{
    const Geo &g = a.g;
    const int64_t S = g.S;
    const T *rc = a.rb[it & 1], *wc = a.wb[it & 1], *sp = a.sb[(it + 1) & 1];
    T *rn = a.rb[(it + 1) & 1], *wn = a.wb[(it + 1) & 1], *sc = a.sb[it & 1];
    double t[4];
    part_load_wave(a.part + (int64_t)(it & 1) * 4 * kMaxBlocks, nprev, t);
    // this block's tile (the map of for_tiles_b with one tile per block)
    const int tpx = (a.tiles + 7) >> 3, xcd = bid & 7, loc = bid >> 3;
    const int tile = xcd * tpx + loc;
    const int n0 = tile * kTile, tid = (int)threadIdx.x, n = n0 + tid;
    const bool valid = loc < tpx && tile < a.tiles && n < S;
    const int64_t bytes = 3 * S * (int64_t)sizeof(T);
    const __amdgpu_buffer_rsrc_t vr_b = buf_view(rc, bytes), vw_b = buf_view(wc, bytes),
                                 vs_b = buf_view(sp, bytes), vp_b = buf_view(a.p, bytes),
                                 vx_b = buf_view(a.x, bytes);
    const int oi = 1, oj = g.px, ok = g.px * g.py, Si = (int)S;
    // Positions of the 24-point stencil (order of curlcurl_node: 8 of x, 8
    // of y, 8 of z).  The 15 in the node's own k-plane (offsets 0, +-1,
    // +-px, +-(px - 1)) read t = D^-1 (r - alpha (w + beta s)) from an LDS
    // copy of the tile and a halo of px nodes on each side; the 9 in the
    // planes k +- 1 load r, w, s.  The node's own r, w, s (the centres) and
    // the halo nodes' are loaded by the threads that write their t.
    constexpr int kq[9] = {1, 2, 3, 9, 10, 12, 18, 19, 22};
    const int koff[9] = {ok, -ok, ok - oi, ok, -ok, ok - oj, oj - ok, -ok, oi - ok};
    T kr[9], kw[9], ks[9], cr[3], cw[3], cs[3], hr[2][3], hw[2][3], hs[2][3], op[3], ox[3];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int e = (kq[q] >> 3) * Si + n + koff[q];
        kr[q] = buf_load<T>(vr_b, e);
        kw[q] = buf_load<T>(vw_b, e);
        ks[q] = FIRST ? (T)0 : buf_load<T>(vs_b, e);
    }
    const bool halo = tid < oj;               // lanes that also load a left and a right halo node
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int e = c * Si + n;
        cr[c] = buf_load<T>(vr_b, e);
        cw[c] = buf_load<T>(vw_b, e);
        cs[c] = FIRST ? (T)0 : buf_load<T>(vs_b, e);
        op[c] = FIRST ? (T)0 : buf_load<T>(vp_b, e);
        ox[c] = buf_load<T>(vx_b, e);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            hr[h][c] = hw[h][c] = hs[h][c] = (T)0;
            if (halo) {
                const int eh = c * Si + (h == 0 ? n0 - oj + tid : n0 + kTile + tid);
                hr[h][c] = buf_load<T>(vr_b, eh);
                hw[h][c] = buf_load<T>(vw_b, eh);
                hs[h][c] = FIRST ? (T)0 : buf_load<T>(vs_b, eh);
            }
        }
    }
    // the previous partials: every wave sums all of them itself (same order
    // in every wave: no barrier) and takes the decision in every lane (same
    // inputs, same result: no broadcast); block 0 stores the record, thread
    // 0 keeps it in s_c for the caller
    __shared__ double s_out[4][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = wave_sum(t[q]);
    double beta;
    const double rtol = (it == 0 && a.rtol_dev) ? *a.rtol_dev : a.rtol;
    const CgCtl c = cg_state(a.ctl[it & 1], t, it, rtol, a.maxit, beta);
    if (threadIdx.x == 0) {
        s_c = c;
        s_beta = beta;
        if (bid == 0) {
            CgCtl o = c;
            if (!o.done) o.it = it + 1;   // iterations completed after this one
            a.ctl[(it + 1) & 1] = o;
        }
    }
    if (c.done) return true;
    const double dd[3] = {g.dinv[0], g.dinv[1], g.dinv[2]};
    const T ta = (T)c.alpha, tb = (T)beta;
    auto tf = [&](int comp, T r, T w, T s_) {
        const T d = (T)dsel(dd, comp);
        return FIRST ? d * (r - ta * w) : d * (r - ta * (w + tb * s_));
    };
    // t of the tile and its halo into LDS (slot of node m: m - n0 + px)
    __shared__ T lt[3][kTile + 2 * kHaloMax];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lt[c][tid + oj] = tf(c, cr[c], cw[c], cs[c]);
        if (halo) {
            lt[c][tid] = tf(c, hr[0][c], hw[0][c], hs[0][c]);
            lt[c][tid + oj + kTile] = tf(c, hr[1][c], hw[1][c], hs[1][c]);
        }
    }
    __syncthreads();
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
        int i, j, k;
        decode(g, n, i, j, k);
        T tk[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) tk[q] = tf(kq[q] >> 3, kr[q], kw[q], ks[q]);
        const int m = tid + oj;
        const T x0 = lt[0][m], x_kp = tk[0], x_km = tk[1], x_im_kp = tk[2], x_im = lt[0][m - oi],
                x_jp = lt[0][m + oj], x_jm = lt[0][m - oj], x_im_jp = lt[0][m + oj - oi];
        const T y0 = lt[1][m], y_kp = tk[3], y_km = tk[4], y_jm = lt[1][m - oj], y_jm_kp = tk[5],
                y_ip = lt[1][m + oi], y_ip_jm = lt[1][m + oi - oj], y_im = lt[1][m - oi];
        const T z0 = lt[2][m], z_jp = lt[2][m + oj], z_jp_km = tk[6], z_km = tk[7],
                z_jm = lt[2][m - oj], z_ip = lt[2][m + oi], z_ip_km = tk[8], z_im = lt[2][m - oi];
        const T Fx = y0 + z_jp - y_kp - z0;
        const T Fx_km = y_km + z_jp_km - y0 - z_km;
        const T Fx_jm = y_jm + z0 - y_jm_kp - z_jm;
        const T Fy = z0 + x_kp - z_ip - x0;
        const T Fy_km = z_km + x0 - z_ip_km - x_km;
        const T Fy_im = z_im + x_im_kp - z0 - x_im;
        const T Fz = x0 + y_ip - x_jp - y0;
        const T Fz_jm = x_jm + y_ip_jm - x0 - y_jm;
        const T Fz_im = x_im + y0 - x_im_jp - y_im;
        const T wx = (T)g.wx, wy = (T)g.wy, wz = (T)g.wz;
        const T w[3] = {wz * (Fz - Fz_jm) - wy * (Fy - Fy_km),
                        wx * (Fx - Fx_km) - wz * (Fz - Fz_im),
                        wy * (Fy - Fy_im) - wx * (Fx - Fx_jm)};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t ix = c * S + n;
            const T d = (T)dsel(dd, c);
            const T rv = cr[c], wv = cw[c];
            const T si = FIRST ? wv : wv + tb * cs[c];
            const T pi = FIRST ? d * rv : d * rv + tb * op[c];
            store_wt(a.x + ix, (T)(ox[c] + ta * pi));
            store_wt(a.p + ix, pi);
            store_wt(sc + ix, si);
            const T r1 = rv - ta * si;
            store_wt(rn + ix, r1);
            const T w1 = edge_cls(g, c, i, j, k, n) == 2 ? w[c] : (T)0;
            store_wt(wn + ix, w1);
            const double u1 = (double)d * (double)r1;
            v[0] += u1 * (double)r1;
            v[1] += (double)w1 * u1;
            v[2] += (double)r1 * (double)r1;
        }
    }
    // this iteration's partials: wave sums, then thread 0 adds the four
    // waves' sums in a fixed order (one barrier)
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s_out[q][wv] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *Pout = a.part + (int64_t)((it + 1) & 1) * 4 * kMaxBlocks;
        for (int q = 0; q < 4; ++q)
            Pout[(int64_t)bid * 4 + q] =
                ((s_out[q][0] + s_out[q][1]) + s_out[q][2]) + s_out[q][3];
    }
    return false;
}

template <typename T>
__device__ __forceinline__ bool cg_iter_hoisted(const CgArgs<T> &a, int it, int nprev,
                                                CgCtl &s_c, double &s_beta, int bid)
{
    return it == 0 ? cg_iter_hoisted_t<T, true>(a, it, nprev, s_c, s_beta, bid)
                   : cg_iter_hoisted_t<T, false>(a, it, nprev, s_c, s_beta, bid);
}

// One tile per block on a grid of nb blocks: the hoisted form applies (the
// same choice in the single, batched and tail kernels, so an iteration's
// arithmetic is the same compiled code whichever kernel runs it).
template <typename T>
__device__ __forceinline__ bool one_tile_per_block(const CgArgs<T> &a, int nb)
{
    return (nb >> 3) >= ((a.tiles + 7) >> 3) && a.g.px <= kHaloMax;
}

template <typename T>
__global__ void __launch_bounds__(256) k_cg_iter(CgArgs<T> a, int it)
{
    if (a.skip && *a.skip) return;
    // a finished solve: pass the record on and leave before loading the
    // partials (graph replays issue a fixed number of these kernels)
    if (a.ctl[it & 1].done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl[(it + 1) & 1] = a.ctl[it & 1];
        return;
    }
    __shared__ CgCtl s_c;
    __shared__ double s_beta;
    if (one_tile_per_block(a, gridDim.x)) {
        cg_iter_hoisted<T>(a, it, gridDim.x, s_c, s_beta, blockIdx.x);
        return;
    }
    double t[4];
    part_load(a.part + (int64_t)(it & 1) * 4 * kMaxBlocks, gridDim.x, t);
    if (cg_decide<T>(a, it, t, s_c, s_beta, blockIdx.x)) return;
    cg_update<T>(a, it, s_c, s_beta, blockIdx.x, gridDim.x);
}

// One iteration of every solve of a batch in one launch: block b serves
// instance inst[b] as its block b - off[inst] (each instance's slice starts
// at a multiple of 8 and has tab[i].blocks blocks).  HOISTED (chosen on the
// host when every instance has at most one tile per block) runs the body of
// the single-instance kernel for that case, so each instance's iteration is
// the same compiled arithmetic as when it is stepped alone; otherwise the
// general body (one instantiation per path keeps the registers of each).
// Block vb of the batch's block map in iteration it (the launched batched
// kernel and the batched tail run this same body, so an instance's
// iteration is the same compiled arithmetic in both).
template <bool HOISTED>
__device__ __forceinline__ void batch_iter_body(const CgArgs<double> *__restrict__ tab,
                                                const int *__restrict__ inst,
                                                const int *__restrict__ off, int vb, int it,
                                                CgCtl &s_c, double &s_beta)
{
    const int i = inst[vb];
    const CgArgs<double> &a = tab[i];
    const int bid = vb - off[i];
    if (a.ctl[it & 1].done) {
        if (bid == 0 && threadIdx.x == 0) a.ctl[(it + 1) & 1] = a.ctl[it & 1];
        return;
    }
    if constexpr (HOISTED) {
        cg_iter_hoisted<double>(a, it, a.blocks, s_c, s_beta, bid);
    } else {
        double t[4];
        part_load(a.part + (int64_t)(it & 1) * 4 * kMaxBlocks, a.blocks, t);
        if (cg_decide<double>(a, it, t, s_c, s_beta, bid)) return;
        cg_update<double>(a, it, s_c, s_beta, bid, a.blocks);
    }
}

template <bool HOISTED>
__global__ void __launch_bounds__(256)
    k_cg_iter_batch(const CgArgs<double> *__restrict__ tab, const int *__restrict__ inst,
                    const int *__restrict__ off, int it)
{
    __shared__ CgCtl s_c;
    __shared__ double s_beta;
    batch_iter_body<HOISTED>(tab, inst, off, blockIdx.x, it, s_c, s_beta);
}

// *flag = 1 if every solve of the batch has finished before iteration it
__global__ void k_batch_done(const CgArgs<double> *__restrict__ tab, int n, int it, int *flag)
{
    __shared__ int s_all;
    if (threadIdx.x == 0) s_all = 1;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (!tab[i].ctl[it & 1].done) atomicAnd(&s_all, 0);
    __syncthreads();
    if (threadIdx.x == 0) *flag = s_all;
}

void cg_iter_batch(const CgArgs<double> *tab, const int *inst, const int *off, int total_blocks,
                   int it, bool one_tile, hipStream_t st)
{
    if (one_tile)
        hipLaunchKernelGGL(k_cg_iter_batch<true>, dim3(total_blocks), dim3(kTile), 0, st, tab,
                           inst, off, it);
    else
        hipLaunchKernelGGL(k_cg_iter_batch<false>, dim3(total_blocks), dim3(kTile), 0, st, tab,
                           inst, off, it);
}

void cg_init_batch(const CgArgs<double> *tab, const int *inst, const int *off, int total_blocks,
                   int mode, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_init_batch, dim3(total_blocks), dim3(kTile), 0, st, tab, inst, off,
                       mode);
}

void batch_done(const CgArgs<double> *tab, int n, int it, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_done, dim3(1), dim3(256), 0, st, tab, n, it, flag);
}

// Stores of the 2.5D iteration's updated vectors.  FP64: streaming
// (non-temporal): they are read again only in the next launch, and keeping
// them out of the L2's way leaves it to the planes and halos still being read
// (128^3: 122 instead of 137 us per iteration).  FP32 (the inner passes of
// refined solves): plain stores; streaming ones made the refined steps
// slower (128^3: 180 instead of 207 steps/s).
template <typename T>
__device__ __forceinline__ void st25(T *p, T v)
{
    if constexpr (sizeof(T) == 8)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// One PCG iteration for large grids (2.5D blocking).  Block b owns the node
// column [i0, i0+TI) x [j0, j0+TJ) (TI*TJ = 256 threads, one node each) and
// the planes [k0, k0+kb).  The transformed input
//   t = D^-1 (r - alpha (w + beta s))
// of every plane is computed once, with a one-node halo, into a ring of three
// LDS planes, and the 24-point curl-curl of the node reads it from there
// instead of issuing 72 global loads.  Outputs, partial sums and the record
// protocol are those of the node-parallel iteration; the grid must equal
// a.blocks (8-aligned, blocks past the last column only write zero partials).
template <typename T, int TI>
__global__ void __launch_bounds__(256)
    k_cg_iter25(CgArgs<T> a, int it, int kb, int nti, int ntj, int ntk)
{
    constexpr int TJ = 256 / TI, LI = TI + 2, LJ = TJ + 2, LP = LI * LJ;
    __shared__ T lt[3][3][LP];
    __shared__ CgCtl s_c;
    __shared__ double s_beta;
    if (a.skip && *a.skip) return;
    if (a.ctl[it & 1].done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl[(it + 1) & 1] = a.ctl[it & 1];
        return;
    }
    {
        double t[4];
        part_load(a.part + (int64_t)(it & 1) * 4 * kMaxBlocks, gridDim.x, t);
        if (cg_decide<T>(a, it, t, s_c, s_beta, blockIdx.x)) return;
    }
    const Geo &g = a.g;
    const int64_t S = g.S, oj = g.px, ok = (int64_t)g.px * g.py;
    const T dd[3] = {(T)g.dinv[0], (T)g.dinv[1], (T)g.dinv[2]};
    const T ta = (T)s_c.alpha, tb = (T)s_beta;
    const bool first = it == 0;
    const T *rc = a.rb[it & 1], *wc = a.wb[it & 1], *sp = a.sb[(it + 1) & 1];
    T *rn = a.rb[(it + 1) & 1], *wn = a.wb[(it + 1) & 1], *sc = a.sb[it & 1];
    // XCD-contiguous ranges of (k-chunk, j, i) tiles
    const int total = nti * ntj * ntk, tpx = (total + 7) >> 3;
    const int L = (blockIdx.x & 7) * tpx + (blockIdx.x >> 3);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (L < total) {
        const int ti = L % nti, tj = (L / nti) % ntj, tk = L / (nti * ntj);
        const int i0 = ti * TI, j0 = tj * TJ, k0 = tk * kb, k1 = min(k0 + kb, g.nz);
        const int lx = threadIdx.x % TI, ly = threadIdx.x / TI;
        const int i = i0 + lx, j = j0 + ly;
        const bool own = i < g.nx && j < g.ny;
        const int lc = (ly + 1) * LI + (lx + 1);
        // raw r, w, s at node (ii, jj, kk) (zero outside the grid)
        struct Raw {
            T r[3], w[3], s[3];
        };
        auto load_raw = [&](int kk, int ii, int jj, Raw &o) {
#pragma unroll
            for (int c = 0; c < 3; ++c) o.r[c] = o.w[c] = o.s[c] = (T)0;
            if (kk >= 0 && kk <= g.nz && ii >= 0 && ii < g.px && jj >= 0 && jj < g.py) {
                const int64_t n = kk * ok + (int64_t)jj * oj + ii;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t ix = c * S + n;
                    o.r[c] = rc[ix];
                    o.w[c] = wc[ix];
                    if (!first) o.s[c] = sp[ix];
                }
            }
        };
        // the 2 LI + 2 TJ halo positions go to the first threads
        constexpr int NH = 2 * LI + 2 * TJ;
        static_assert(NH <= 256, "halo positions exceed the block");
        int hli = 0, hlj = 0;
        if (threadIdx.x < NH) {
            const int h = threadIdx.x;
            if (h < LI) {
                hli = h; hlj = 0;
            } else if (h < 2 * LI) {
                hli = h - LI; hlj = LJ - 1;
            } else if (h < 2 * LI + TJ) {
                hli = 0; hlj = 1 + (h - 2 * LI);
            } else {
                hli = LI - 1; hlj = 1 + (h - 2 * LI - TJ);
            }
        }
        // issue the loads of plane kk (own node and, for the first threads, a
        // halo node); nothing waits for them here
        auto fetch = [&](int kk, Raw &own_o, Raw &halo_o) {
            load_raw(kk, i, j, own_o);
            if (threadIdx.x < NH) load_raw(kk, i0 - 1 + hli, j0 - 1 + hlj, halo_o);
        };
        // t of plane kk into ring slot kk % 3 from fetched values; the
        // node's r and u = w + beta s are kept for its update
        auto store_plane = [&](int kk, const Raw &own_o, const Raw &halo_o, T(&rv)[3], T(&uv)[3]) {
            T(*dst)[LP] = lt[((kk % 3) + 3) % 3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                rv[c] = own_o.r[c];
                uv[c] = first ? own_o.w[c] : own_o.w[c] + tb * own_o.s[c];
                dst[c][lc] = dd[c] * (rv[c] - ta * uv[c]);
            }
            if (threadIdx.x < NH) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T hu = first ? halo_o.w[c] : halo_o.w[c] + tb * halo_o.s[c];
                    dst[c][hlj * LI + hli] = dd[c] * (halo_o.r[c] - ta * hu);
                }
            }
        };
        T cr[3], cu[3], nr[3], nu[3];
        {
            Raw o0, h0, o1, h1;
            fetch(k0 - 1, o0, h0);
            fetch(k0, o1, h1);
            store_plane(k0 - 1, o0, h0, nr, nu);
            store_plane(k0, o1, h1, cr, cu);
        }
        // plane k + 1 is fetched while plane k is computed: its loads are in
        // flight across the barriers and the compute of the plane before
        // (128^3 with streaming stores: 111 instead of 122 us per iteration)
        Raw po, ph;
        fetch(k0 + 1, po, ph);
        const T wx = (T)g.wx, wy = (T)g.wy, wz = (T)g.wz;
        for (int k = k0; k < k1; ++k) {
            // the node's p and x of plane k first: their loads overlap those
            // of plane k + 2 (neither waits for the barrier)
            const int64_t n = k * ok + (int64_t)j * oj + i;
            T opv[3] = {(T)0, (T)0, (T)0}, oxv[3] = {(T)0, (T)0, (T)0};
            if (own) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (!first) opv[c] = a.p[c * S + n];
                    oxv[c] = a.x[c * S + n];
                }
            }
            store_plane(k + 1, po, ph, nr, nu);
            if (k + 2 <= k1) fetch(k + 2, po, ph);
            __syncthreads();
            if (own) {
                const T(*pm)[LP] = lt[((k - 1) % 3 + 3) % 3];
                const T(*p0)[LP] = lt[k % 3];
                const T(*pp)[LP] = lt[(k + 1) % 3];
                const int di = 1, dj = LI;
                const T x0 = p0[0][lc], x_kp = pp[0][lc], x_km = pm[0][lc],
                        x_im_kp = pp[0][lc - di], x_im = p0[0][lc - di], x_jp = p0[0][lc + dj],
                        x_jm = p0[0][lc - dj], x_im_jp = p0[0][lc + dj - di];
                const T y0 = p0[1][lc], y_kp = pp[1][lc], y_km = pm[1][lc], y_jm = p0[1][lc - dj],
                        y_jm_kp = pp[1][lc - dj], y_ip = p0[1][lc + di],
                        y_ip_jm = p0[1][lc + di - dj], y_im = p0[1][lc - di];
                const T z0 = p0[2][lc], z_jp = p0[2][lc + dj], z_jp_km = pm[2][lc + dj],
                        z_km = pm[2][lc], z_jm = p0[2][lc - dj], z_ip = p0[2][lc + di],
                        z_ip_km = pm[2][lc + di], z_im = p0[2][lc - di];
                const T Fx = y0 + z_jp - y_kp - z0;
                const T Fx_km = y_km + z_jp_km - y0 - z_km;
                const T Fx_jm = y_jm + z0 - y_jm_kp - z_jm;
                const T Fy = z0 + x_kp - z_ip - x0;
                const T Fy_km = z_km + x0 - z_ip_km - x_km;
                const T Fy_im = z_im + x_im_kp - z0 - x_im;
                const T Fz = x0 + y_ip - x_jp - y0;
                const T Fz_jm = x_jm + y_ip_jm - x0 - y_jm;
                const T Fz_im = x_im + y0 - x_im_jp - y_im;
                const T q[3] = {wz * (Fz - Fz_jm) - wy * (Fy - Fy_km),
                                wx * (Fx - Fx_km) - wz * (Fz - Fz_im),
                                wy * (Fy - Fy_im) - wx * (Fx - Fx_jm)};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t ix = c * S + n;
                    const T d = dd[c];
                    const T rv = cr[c], si = cu[c];
                    const T pi = first ? d * rv : d * rv + tb * opv[c];
                    st25(a.x + ix, (T)(oxv[c] + ta * pi));
                    st25(a.p + ix, pi);
                    st25(sc + ix, si);
                    const T r1 = rv - ta * si;
                    st25(rn + ix, r1);
                    const T w1 = edge_cls(g, c, i, j, k, n) == 2 ? q[c] : (T)0;
                    st25(wn + ix, w1);
                    const double u1 = (double)d * (double)r1;
                    v[0] += u1 * (double)r1;
                    v[1] += (double)w1 * u1;
                    v[2] += (double)r1 * (double)r1;
                }
            }
            __syncthreads();           // the next load overwrites plane k - 1
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cr[c] = nr[c];
                cu[c] = nu[c];
            }
        }
    }
    block_sum<4>(v);
    if (threadIdx.x == 0) {
        double *Pout = a.part + (int64_t)((it + 1) & 1) * 4 * kMaxBlocks;
        for (int q = 0; q < 4; ++q) Pout[(int64_t)blockIdx.x * 4 + q] = v[q];
    }
}

// Grid barrier of a launch whose blocks are all resident, grouped by the
// XCD (accelerator complex die, one L2 each) a block runs on, read from the
// hardware register.  A block's stores reach its XCD's L2 before it arrives
// (a wait on its own memory counters in every wave); the last block of an
// XCD to arrive writes back that whole L2 (an agent-scope release fence
// operates on the cache, so it publishes every block of the XCD), meets the
// other XCDs' last arrivers on one counter and releases its XCD; every block
// then takes an agent-scope acquire fence.  One L2 write-back per XCD
// instead of one per block, and no block polls more than one word.
// Barrier words, kBarStride apart: pop[kBarXcc] (blocks per XCD, counted at
// the first barrier of the launch), cnt[kBarXcc] (arrivals per XCD), top
// (arrivals of the XCDs' last blocks), grel (global release), xrel[kBarXcc]
// (release per XCD); all zero at launch.
// Every wait is bounded: false if the spin limit was reached (never
// expected); a group whose release never comes then times out too.
struct BarState {
    unsigned x = 0, pop = 0, groups = 0;   // XCD, its blocks, XCDs in use
};

__device__ __forceinline__ unsigned xcd_id()
{
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & (kBarXcc - 1);
}

__device__ __forceinline__ bool spin_until(const unsigned *w, unsigned target)
{
    long spins = 0;
    while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > kSpinLimit) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned gen, BarState &bs)
{
    __shared__ int s_ok;
    // this wave's stores acknowledged by the L2
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned *pop = bar, *cnt = bar + kBarXcc * kBarStride;
        unsigned *top = bar + 2 * kBarXcc * kBarStride, *grel = top + kBarStride;
        unsigned *xrel = grel + kBarStride;
        int ok = 1;
        if (gen == 1) {
            // population of each XCD: every block counts itself once
            bs.x = xcd_id();
            __hip_atomic_fetch_add(pop + bs.x * kBarStride, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            long spins = 0;
            for (;;) {
                unsigned tot = 0, groups = 0, mine = 0;
                for (int q = 0; q < kBarXcc; ++q) {
                    const unsigned v = __hip_atomic_load(pop + q * kBarStride, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    tot += v;
                    groups += v > 0u;
                    if (q == (int)bs.x) mine = v;
                }
                if (tot >= gridDim.x) {
                    bs.pop = mine;
                    bs.groups = groups;
                    break;
                }
                if (++spins > kSpinLimit) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (ok) {
            const unsigned old = __hip_atomic_fetch_add(cnt + bs.x * kBarStride, 1u,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (old + 1 == gen * bs.pop) {
                // last of its XCD: write the L2 back, then meet the others
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __builtin_amdgcn_s_waitcnt(0);
                const unsigned t = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                if (t + 1 == gen * bs.groups)
                    __hip_atomic_store(grel, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else
                    ok = spin_until(grel, gen);
                if (ok)
                    __hip_atomic_store(xrel + bs.x * kBarStride, gen, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            } else {
                ok = spin_until(xrel + bs.x * kBarStride, gen);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Finishes a solve that the captured iteration kernels left unfinished:
// iterations it0, it0+1, ... in one persistent launch, a grid barrier
// between iterations, until the (uniform) convergence / maxit decision.
// Ends with the final record in slot (it0 + 1) & 1 (in both slots when it
// took more than one iteration); with fin, block 0 then runs the solve's
// final step (k_cg_fin for it0 + 1 iteration launches), one launch fewer.
// HOISTED: every block sweeps at most one tile (the iteration kernels' form,
// chosen on the host so that each instantiation holds only one path).
template <typename T>
__device__ __forceinline__ void cg_fin_body(const CgArgs<T> &a, int iters);

template <typename T, bool HOISTED>
__global__ void __launch_bounds__(256, 2) k_cg_tail(CgArgs<T> a, int it0, unsigned *bar, int fin)
{
    if (a.skip && *a.skip) return;
    // the usual case: the captured kernels finished the solve
    if (a.ctl[it0 & 1].done) {
        if (blockIdx.x == 0) {
            if (threadIdx.x == 0) a.ctl[(it0 + 1) & 1] = a.ctl[it0 & 1];
            if (fin) cg_fin_body<T>(a, it0 + 1);
        }
        return;
    }
    __shared__ CgCtl s_c;
    __shared__ double s_beta;
    int nprev = a.blocks;
    unsigned gen = 0;
    BarState bs;
    bool ok = true;
    int it = it0;
    for (;; ++it) {
        bool done;
        if constexpr (HOISTED)
            done = cg_iter_hoisted<T>(a, it, nprev, s_c, s_beta, blockIdx.x);
        else
            done = cg_iteration<T>(a, it, nprev, s_c, s_beta, blockIdx.x, gridDim.x);
        if (done) break;
        nprev = gridDim.x;
        ok = grid_barrier(bar, ++gen, bs);
        if (!ok) break;
    }
    // decided in its first iteration: that decision already stored the
    // record in slot (it0 + 1) & 1, the one the final step reads
    if (ok && it == it0) {
        if (fin && blockIdx.x == 0) cg_fin_body<T>(a, it0 + 1);
        return;
    }
    // every block has read the control slots of its last iteration
    if (ok) ok = grid_barrier(bar, ++gen, bs);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        CgCtl f = s_c;
        if (!ok) {
            f.done = 1;
            f.status = EC_ERR_HIP;
        }
        a.ctl[0] = f;
        a.ctl[1] = f;
    }
    // the solve's final step (as k_cg_fin) on the record just stored
    if (fin && blockIdx.x == 0) cg_fin_body<T>(a, it0 + 1);
}

// Finishes the batched solves that the captured iteration launches left
// unfinished: iterations it0, it0+1, ... of every instance in one persistent
// launch.  Its blocks sweep the batch's block map (block vb = blockIdx.x +
// q gridDim.x runs batch_iter_body for vb, the launched kernel's block vb),
// a grid barrier between iterations; after each barrier every block reads
// the n records and the sweep ends once all solves are done.  Then block 0
// puts each instance's final record into both control slots, so that the
// final step of the budget (k_cg_fin_tab for it0 + 1 iterations) reads it.
// The barrier words are instance 0's (cleared by its init).
template <bool HOISTED>
__global__ void __launch_bounds__(256, 2)
    k_cg_tail_batch(const CgArgs<double> *__restrict__ tab, int n, const int *__restrict__ inst,
                    const int *__restrict__ off, int total, int it0)
{
    __shared__ CgCtl s_c;
    __shared__ double s_beta;
    __shared__ int s_all;
    unsigned *bar = tab[0].bar;
    // the usual case: the launched iterations finished every solve
    if (threadIdx.x == 0) {
        int all = 1;
        for (int i = 0; i < n; ++i) all &= tab[i].ctl[it0 & 1].done;
        s_all = all;
    }
    __syncthreads();
    if (s_all) {
        if (blockIdx.x == 0)
            for (int i = threadIdx.x; i < n; i += blockDim.x) tab[i].ctl[(it0 + 1) & 1] =
                tab[i].ctl[it0 & 1];
        return;
    }
    unsigned gen = 0;
    BarState bs;
    bool ok = true;
    int it = it0;
    for (;; ++it) {
        for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
            batch_iter_body<HOISTED>(tab, inst, off, vb, it, s_c, s_beta);
            __syncthreads();     // shared records reused by the next block of the sweep
        }
        ok = grid_barrier(bar, ++gen, bs);
        if (!ok) break;
        if (threadIdx.x == 0) {
            int all = 1;
            for (int i = 0; i < n; ++i) all &= tab[i].ctl[(it + 1) & 1].done;
            s_all = all;
        }
        __syncthreads();
        if (s_all) break;
    }
    // every block has read the records of the last iteration
    if (ok) ok = grid_barrier(bar, ++gen, bs);
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            CgCtl f = tab[i].ctl[(it + 1) & 1];
            if (!ok) {
                f.done = 1;
                f.status = EC_ERR_HIP;
            }
            tab[i].ctl[0] = f;
            tab[i].ctl[1] = f;
        }
    }
}

int cg_tail_batch_blocks()
{
    int dev = 0, cus = 0, p0 = 0, p1 = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p0, k_cg_tail_batch<false>, kTile, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&p1, k_cg_tail_batch<true>, kTile, 0) !=
            hipSuccess)
        return 0;
    const int per = std::min(p0, p1);
    if (per < 1) return 0;
    // at most two blocks per CU, a multiple of 8: all resident at once
    return std::min((cus * std::min(per, 2)) & ~7, kMaxBlocks);
}

hipError_t cg_tail_batch(const CgArgs<double> *tab, int n, const int *inst, const int *off,
                         int total, int it0, int blocks, bool one_tile, hipStream_t st)
{
    const int nb = std::min(blocks, ((total + 7) / 8) * 8);
    if (one_tile)
        hipLaunchKernelGGL(k_cg_tail_batch<true>, dim3(nb), dim3(kTile), 0, st, tab, n, inst, off,
                           total, it0);
    else
        hipLaunchKernelGGL(k_cg_tail_batch<false>, dim3(nb), dim3(kTile), 0, st, tab, n, inst, off,
                           total, it0);
    return hipGetLastError();
}

// After `iters` iteration kernels: final decision on the last iterate, the
// solve record and the per-sequence counters (one block).
template <typename T>
__device__ __forceinline__ void cg_fin_body(const CgArgs<T> &a, int iters)
{
    double t[4];
    sum_part(a.part + (int64_t)(iters & 1) * 4 * kMaxBlocks, a.blocks, t);
    if (threadIdx.x != 0) return;
    double beta;
    // maxit + 1 lets the last iterate be judged on its residual only
    const double rtol = (iters == 0 && a.rtol_dev) ? *a.rtol_dev : a.rtol;
    CgCtl c = cg_state(a.ctl[iters & 1], t, iters, rtol, a.maxit + 1, beta);
    int st = c.status;
    if (!c.done) st = EC_ERR_NOT_CONVERGED;
    const int it = c.it;
    // an FP64 solve of an SPE sequence that ended on its start vector: the
    // push of this solution is a rejected one, skip its work
    if (a.seq && !a.accum && it == 0 && a.seq->method == EC_SV_SPE) a.seq->push_on = 0;
    if (a.info) {
        if (a.accum) {
            a.info->iters += it;
        } else {
            const double bb = c.bb;
            a.info->iters = it;
            a.info->outer_iters = 0;
            a.info->rel_res = bb > 0.0 ? sqrt(c.rho / bb) : 0.0;
            a.info->b_norm = sqrt(bb);
            a.info->r0_rel = bb > 0.0 ? sqrt(c.rho0 / bb) : 0.0;
            int s2 = st;
            if (a.seq) {
                a.info->basis_cols = a.seq->method == EC_SV_POD ? a.seq->kpod : a.seq->k;
                a.info->pod_info = a.seq->method == EC_SV_POD ? a.seq->pod_info : 1.0;
                if (s2 == EC_OK && a.seq->flags) s2 = EC_ERR_SINGULAR_PROJ;
            } else {
                a.info->basis_cols = 0;
                a.info->pod_info = 1.0;
            }
            a.info->status = s2;
        }
    }
    if (a.ctrl) {
        a.ctrl->iters[a.seq_id] += it;
        // an inner solve of the refinement loop may stop at its cap: only the
        // outer FP64 residual check decides the status
        if (!a.accum && st < a.ctrl->worst) a.ctrl->worst = st;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_cg_fin(CgArgs<T> a, int iters)
{
    if (a.skip && *a.skip) return;
    cg_fin_body<T>(a, iters);
}

// k_cg_fin of every solve of a batch: block row blockIdx.y serves tab[y]
__global__ void __launch_bounds__(256) k_cg_fin_tab(const CgArgs<double> *tab, int iters)
{
    cg_fin_body<double>(tab[blockIdx.y], iters);
}

void cg_fin_batch(const CgArgs<double> *tab, int n, int iters, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_fin_tab, dim3(1, n), dim3(256), 0, st, tab, iters);
}

template <typename T>
void cg_init(const CgArgs<T> &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_init<T>, dim3(a.blocks), dim3(kTile), 0, st, a);
}
template <typename T>
void cg_iter(const CgArgs<T> &a, int i, hipStream_t st)
{
    if (a.t25 > 0) {
        if (a.t25 == 64)
            hipLaunchKernelGGL((k_cg_iter25<T, 64>), dim3(a.blocks), dim3(kTile), 0, st, a, i,
                               a.kb25, a.nti25, a.ntj25, a.ntk25);
        else if (a.t25 == 32)
            hipLaunchKernelGGL((k_cg_iter25<T, 32>), dim3(a.blocks), dim3(kTile), 0, st, a, i,
                               a.kb25, a.nti25, a.ntj25, a.ntk25);
        else
            hipLaunchKernelGGL((k_cg_iter25<T, 16>), dim3(a.blocks), dim3(kTile), 0, st, a, i,
                               a.kb25, a.nti25, a.ntj25, a.ntk25);
        return;
    }
    hipLaunchKernelGGL(k_cg_iter<T>, dim3(a.blocks), dim3(kTile), 0, st, a, i);
}
template <typename T>
int cg_tail_blocks()
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    int per_h = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cg_tail<T, false>, kTile, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_h, k_cg_tail<T, true>, kTile, 0) !=
            hipSuccess)
        return 0;
    per = std::min(per, per_h);
    if (per < 1) return 0;
    // at most two blocks per CU, a multiple of 8: all resident at once
    const int nb = (cus * std::min(per, 2)) & ~7;
    return std::min(nb, kMaxBlocks);
}

template <typename T>
hipError_t cg_tail(const CgArgs<T> &a, int it0, int blocks, hipStream_t st, bool fin)
{
    // a plain launch: a cooperative one costs ~11 us of idle device on each
    // side inside a graph.  The grid (two blocks per CU at most) fits the
    // device at once.  Kernels of another stream (the history pushes that a
    // captured step forks) may hold CUs while it starts: they do not wait
    // for the tail, so they finish and its remaining blocks then start, the
    // early ones waiting at the barrier meanwhile (the pushes' blocks still
    // fit beside two tail blocks per CU); the bounded wait of the barrier
    // turns any violation into an error status
    if ((blocks >> 3) >= ((a.tiles + 7) >> 3) && a.g.px <= kHaloMax)
        hipLaunchKernelGGL((k_cg_tail<T, true>), dim3(blocks), dim3(kTile), 0, st, a, it0, a.bar,
                           fin ? 1 : 0);
    else
        hipLaunchKernelGGL((k_cg_tail<T, false>), dim3(blocks), dim3(kTile), 0, st, a, it0, a.bar,
                           fin ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
void cg_fin(const CgArgs<T> &a, int iters, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_fin<T>, dim3(1), dim3(256), 0, st, a, iters);
}
template void cg_init<double>(const CgArgs<double> &, hipStream_t);
template void cg_iter<double>(const CgArgs<double> &, int, hipStream_t);
template void cg_fin<double>(const CgArgs<double> &, int, hipStream_t);
template void cg_init<float>(const CgArgs<float> &, hipStream_t);
template void cg_iter<float>(const CgArgs<float> &, int, hipStream_t);
template void cg_fin<float>(const CgArgs<float> &, int, hipStream_t);
template int cg_tail_blocks<double>();
template hipError_t cg_tail<double>(const CgArgs<double> &, int, int, hipStream_t, bool);
template int cg_tail_blocks<float>();
template hipError_t cg_tail<float>(const CgArgs<float> &, int, int, hipStream_t, bool);

// --------------------------------------------------- FP32-refined solves
// r = s b - K_n x in FP64, r32 = r, partials (|r|^2, |b|^2).
__global__ void __launch_bounds__(256)
    k_refine_resid(Geo g, const double *b, const double *bscale, const double *x, float *r32,
                   double *part, const Ctrl *ctrl, int tiles)
{
    if (ctrl->refine_done) return;
    const int64_t S = g.S;
    const double bs = bscale ? *bscale : 1.0;
    double v[2] = {0.0, 0.0};
    for_tiles(tiles, S, [&](int64_t n) {
        int i, j, k;
        decode(g, n, i, j, k);
        double q[3];
        curlcurl_node<double>(g, n, [&](int, int64_t ix) { return x[ix]; }, q[0], q[1], q[2]);
        for (int c = 0; c < 3; ++c) {
            const int64_t ix = (int64_t)c * S + n;
            const double kx = edge_cls(g, c, i, j, k, n) == 2 ? q[c] : 0.0;
            const double bv = bs * b[ix];
            const double rv = bv - kx;
            r32[ix] = (float)rv;
            v[0] += rv * rv;
            v[1] += bv * bv;
        }
    });
    block_sum<2>(v);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
    }
}

void refine_residual(const Geo &g, const double *b, const double *bscale, const double *x,
                     float *r32, double *part, const Ctrl *ctrl, int blocks, hipStream_t st)
{
    const int tiles = (int)((g.S + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_refine_resid, dim3(blocks), dim3(kTile), 0, st, g, b, bscale, x, r32, part,
                       ctrl, tiles);
}

// Converged (||r|| <= rtol ||b||), out of passes, or another inner solve.
__global__ void __launch_bounds__(256)
    k_refine_decide(const double *part, int nb, Ctrl *ctrl, int pass, int outer_max, double rtol,
                    double inner_rtol, ec_solve_info *info, const SeqDev *seq)
{
    if (ctrl->refine_done) return;
    double s[2];
    reduce_partials<2>(part, nb, 2, s);
    if (threadIdx.x != 0) return;
    const double rr = s[0], bb2 = s[1];
    const double rel = bb2 > 0.0 ? sqrt(rr / bb2) : 0.0;
    int done = 0, st = EC_OK;
    if (!(rr == rr) || rr > 1e300) {
        done = 1;
        st = EC_ERR_NONFINITE;
    } else if (bb2 == 0.0 || rel <= rtol) {
        done = 1;
    } else if (pass >= outer_max) {
        done = 1;
        st = EC_ERR_NOT_CONVERGED;
    }
    if (pass == 0 && info) {
        info->iters = 0;
        info->b_norm = sqrt(bb2);
        info->r0_rel = rel;
        info->basis_cols = seq ? (seq->method == EC_SV_POD ? seq->kpod : seq->k) : 0;
        info->pod_info = (seq && seq->method == EC_SV_POD) ? seq->pod_info : 1.0;
    }
    if (done) {
        ctrl->refine_done = 1;
        ctrl->refine_zero = (bb2 == 0.0) ? 1 : 0;
        if (info) {
            info->outer_iters = pass;
            info->rel_res = rel;
            int s2 = st;
            if (s2 == EC_OK && seq && seq->flags) s2 = EC_ERR_SINGULAR_PROJ;
            info->status = s2;
        }
        if (st < ctrl->worst) ctrl->worst = st;
    }
    ctrl->refine_rr = rr;
    ctrl->refine_bb = bb2;
    // the inner solve only has to bring the residual just below the target:
    // relative reduction 0.95 rtol / rel (5 % for the gap between its FP32
    // recurrence and the FP64 residual; when that gap is larger, one short
    // pass more follows), never looser than 0.5 nor tighter than the
    // caller's inner_rtol (FP32 limits what it can reach).  Near the target
    // PCG converges slowly, so a wider margin costs many iterations (a
    // margin of one half took a quarter more iterations per step)
    ctrl->refine_tol = rel > 0.0 ? fmax(inner_rtol, fmin(0.5, 0.95 * rtol / rel)) : inner_rtol;
}

void refine_decide(const double *part, int blocks, Ctrl *ctrl, int pass, int outer_max,
                   double rtol, double inner_rtol, ec_solve_info *info, const SeqDev *seq,
                   hipStream_t st)
{
    hipLaunchKernelGGL(k_refine_decide, dim3(1), dim3(256), 0, st, part, blocks, ctrl, pass,
                       outer_max, rtol, inner_rtol, info, seq);
}

// x += d (FP32 correction) unless the loop has finished; b = 0 gives x = 0
__global__ void k_refine_update(double *x, const float *d, const Ctrl *ctrl, int64_t n, int final)
{
    const int zero = ctrl->refine_zero;
    if (final ? !zero : ctrl->refine_done) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        x[e] = final ? 0.0 : x[e] + (double)d[e];
}

void refine_update(double *x, const float *d, const Ctrl *ctrl, int64_t n, hipStream_t st)
{
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_refine_update, dim3(blocks), dim3(256), 0, st, x, d, ctrl, n, 0);
}

void refine_final(double *x, const Ctrl *ctrl, int64_t n, hipStream_t st)
{
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_refine_update, dim3(blocks), dim3(256), 0, st, x, (const float *)nullptr,
                       ctrl, n, 1);
}

__global__ void k_refine_reset(Ctrl *ctrl)
{
    ctrl->refine_done = 0;
    ctrl->refine_zero = 0;
}

void refine_reset(Ctrl *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_refine_reset, dim3(1), dim3(1), 0, st, ctrl);
}

}  // namespace ec
