// ec_basis.hip -- start vectors of Sec. III on gfx950.
//
// SPE (eq. 10): per right-hand-side sequence an orthogonal basis q of the
// span of the last m accepted solutions, kept with its K_n products (the
// cascaded reuse of the paper: only a new column needs an SpMV), and
// x0 = q (q^T K_n q)^{-1} q^T b.  New solutions are orthogonalised by two
// classical Gram-Schmidt passes; the oldest solution leaves the window by a
// Givens downdate of the window's triangular coordinates, which rotates the
// basis (and its K_n products) in place.
// POD (eqs. 11-14): a ring of N_POD snapshots X with K_n X; the snapshot Gram
// matrix X^T X = V Sigma^2 V^T gives the left singular vectors u_j =
// X v_j / sigma_j (method of snapshots), truncated by sigma_j >= eps sigma_1
// and at most kmax modes; eq. (13) is reported; x0 from eq. (14).
//
// The tall-skinny products run on the FP64 matrix cores and leave one row of
// partial sums per block; the small dense step of the sequence (OP_* codes)
// that follows reduces the rows in a fixed order, in a one-block kernel or,
// for the coefficient steps of a push, in every block of the kernel that
// applies the coefficients.
#include <math.h>

#include "ec_device.h"

namespace ec {

typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int K = kMaxWin;
constexpr int KC = EC_MAX_WINDOW + 1;     // columns a basis can hold
// threads of the tall-skinny kernels: 16 waves per block (four per SIMD)
// hide the memory latency of these streaming passes; the grid stays at
// kMdBlocks blocks, so the partial rows keep their count
constexpr int kMdThreads = 1024;
constexpr int kMdWaves = kMdThreads / 64;

// ------------------------------------------------ small dense primitives
// All threads of the block call these (uniform barriers); serial parts run
// on thread 0, parallel loops stride over the block.

// value of v in lane l (l the same in every lane): two scalar lane reads
__device__ __forceinline__ double lane_read(double v, int l)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The factorisation half of chol_wave below, statement for statement, for
// a factor that is stored and used later (same operations, same factor).
// Cholesky factorisation of H (n x n, leading dimension K, n <= NM) by wave
// 0, lane r holding row r of the factor in a[] (no block barrier inside):
// right-looking, column j scaled by the pivot's square root, then the
// trailing lower triangle updated.  bad: a pivot not positive relative to
// the largest diagonal entry.
template <int NM>
__device__ __forceinline__ void chol_factor_regs(const double *H, int n, double (&a)[NM], int &bad,
                                                 double hscale)
{
    const int r = threadIdx.x;
#pragma unroll
    for (int c = 0; c < NM; ++c) a[c] = (r < n && c <= r) ? H[r * K + c] : 0.0;
    double dg = 0.0;
#pragma unroll
    for (int c = 0; c < NM; ++c)
        if (c == r) dg = a[c];
    double dmax = r < n ? fabs(dg) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
    dmax = fmax(dmax, hscale);
    bad = 0;
#pragma unroll
    for (int j = 0; j < NM; ++j) {
        if (j < n) {
            const double d = lane_read(a[j], j);
            if (!(d > 1e-14 * dmax)) bad = 1;
            const double ljj = d > 0.0 ? sqrt(d) : 1.0;
            if (r == j) a[j] = ljj;
            else if (r > j) a[j] /= ljj;
#pragma unroll
            for (int c = j + 1; c < NM; ++c) {
                if (c < n) {
                    const double lcj = lane_read(a[j], c);
                    if (r >= c) a[c] -= a[j] * lcj;
                }
            }
        }
    }
}

// Cholesky solve H y = g (n x n, leading dimension K, n <= NM) by wave 0,
// lane r holding row r of the factor in registers (no block barrier inside):
// right-looking, column j scaled by the pivot's square root, then the
// trailing lower triangle updated; forward substitution by columns,
// backward by rows.  Sets *bad when a pivot is not positive relative to the
// largest diagonal entry.  y: n values (shared memory).
template <int NM>
__device__ __forceinline__ void chol_wave(const double *H, double *y, const double *gv, int n,
                                          int *bad_out, double hscale)
{
    const int r = threadIdx.x;
    double a[NM];
#pragma unroll
    for (int c = 0; c < NM; ++c) a[c] = (r < n && c <= r) ? H[r * K + c] : 0.0;
    double gr = r < n ? gv[r] : 0.0;
    double dg = 0.0;
#pragma unroll
    for (int c = 0; c < NM; ++c)
        if (c == r) dg = a[c];
    double dmax = r < n ? fabs(dg) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
    dmax = fmax(dmax, hscale);
    int bad = 0;
#pragma unroll
    for (int j = 0; j < NM; ++j) {
        if (j < n) {
            const double d = lane_read(a[j], j);
            if (!(d > 1e-14 * dmax)) bad = 1;
            const double ljj = d > 0.0 ? sqrt(d) : 1.0;
            if (r == j) a[j] = ljj;
            else if (r > j) a[j] /= ljj;
#pragma unroll
            for (int c = j + 1; c < NM; ++c) {
                if (c < n) {
                    const double lcj = lane_read(a[j], c);
                    if (r >= c) a[c] -= a[j] * lcj;
                }
            }
        }
    }
    // L z = g: z_j leaves lane j, the rows below subtract L[r][j] z_j
    double z[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) {
        z[j] = 0.0;
        if (j < n) {
            z[j] = lane_read(gr, j) / lane_read(a[j], j);
            if (r > j) gr -= a[j] * z[j];
        }
    }
    // L^T y = z, rows from the last: y_i = (z_i - sum_{j>i} L[j][i] y_j) / L[i][i]
#pragma unroll
    for (int i = NM - 1; i >= 0; --i) {
        if (i < n) {
            double t = z[i];
#pragma unroll
            for (int j = i + 1; j < NM; ++j)
                if (j < n) t -= lane_read(a[i], j) * z[j];
            z[i] = t / lane_read(a[i], i);
        }
    }
    if (r == 0) {
#pragma unroll
        for (int c = 0; c < NM; ++c)
            if (c < n) y[c] = z[c];
        *bad_out = bad;
    }
}

// The same factorisation for any n <= K with the factor in shared memory L
// (leading dimension K), serial parts on thread 0, block barriers between
// the steps.
__device__ __noinline__ int chol_shared(const double *H, double *L, double *y, const double *gv,
                                        int n, double hscale)
{
    __shared__ int s_bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) s_bad = 0;
    for (int t = tid; t < n * n; t += nt) {
        const int r = t / n, c = t - r * n;
        L[r * K + c] = H[r * K + c];
    }
    __syncthreads();
    double dmax = hscale;
    for (int i = 0; i < n; ++i) dmax = fmax(dmax, fabs(L[i * K + i]));
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double d = L[j * K + j];
            if (!(d > 1e-14 * dmax)) s_bad = 1;
            L[j * K + j] = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double ljj = L[j * K + j];
        for (int i = j + 1 + tid; i < n; i += nt) L[i * K + j] /= ljj;
        __syncthreads();
        const int m = n - j - 1;
        for (int t = tid; t < m * m; t += nt) {
            const int r = j + 1 + t / m, c = j + 1 + t % m;
            if (c <= r) L[r * K + c] -= L[r * K + j] * L[c * K + j];
        }
        __syncthreads();
    }
    if (tid == 0) {
        for (int i = 0; i < n; ++i) {
            double s = gv[i];
            for (int j = 0; j < i; ++j) s -= L[i * K + j] * y[j];
            y[i] = s / L[i * K + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int j = i + 1; j < n; ++j) s -= L[j * K + i] * y[j];
            y[i] = s / L[i * K + i];
        }
    }
    __syncthreads();
    return s_bad;
}

// Cholesky solve H y = g (n x n, leading dimension K, n <= K); false if H is
// not numerically positive definite.  All threads of the block call it.
// Windows of up to kCholReg columns (the usual case) factor in registers on
// wave 0; larger ones in shared memory L.
constexpr int kCholReg = 12;
__device__ bool chol_solve(const double *H, double *L, double *y, const double *gv, int n,
                           double hscale)
{
    __shared__ int s_bad;
    if (n > kCholReg) return chol_shared(H, L, y, gv, n, hscale) == 0;
    if (threadIdx.x < 64) chol_wave<kCholReg>(H, y, gv, n, &s_bad, hscale);
    __syncthreads();
    return s_bad == 0;
}

// The SPE start's solve H y = g from the factor that the last push stored
// (SeqDev::L), copied to shared memory Lsh (leading dimension K) and
// substituted on thread 0 in the operation order of chol_wave's
// substitutions; false if that factor is not current (then chol_solve).
__device__ __forceinline__ bool chol_solve_stored(const SeqDev *sq, double *Lsh, double *y,
                                                  const double *gv, int n, bool *good)
{
    __shared__ int s_use, s_bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) {
        s_use = n <= kCholReg && sq->L_ver == sq->H_ver;
        s_bad = sq->chol_bad;
    }
    __syncthreads();
    if (!s_use) return false;
    for (int t = tid; t < n * n; t += nt) {
        const int r = t / n, c = t - r * n;
        Lsh[r * K + c] = c <= r ? sq->L[r * K + c] : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        for (int i = 0; i < n; ++i) {
            double t = gv[i];
            for (int j = 0; j < i; ++j) t -= Lsh[i * K + j] * y[j];
            y[i] = t / Lsh[i * K + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double t = y[i];
            for (int j = i + 1; j < n; ++j) t -= Lsh[j * K + i] * y[j];
            y[i] = t / Lsh[i * K + i];
        }
    }
    __syncthreads();
    *good = s_bad == 0;
    return true;
}

// Factor H of an SPE sequence into SeqDev::L when a push changed it (wave 0
// of one block; windows of up to kCholReg columns).
__device__ __forceinline__ void chol_store(SeqDev *sq)
{
    if (threadIdx.x >= 64) return;
    const int n = sq->k, hv = sq->H_ver;
    if (sq->L_ver == hv || n < 1 || n > kCholReg) return;
    double a[kCholReg];
    int bad;
    chol_factor_regs<kCholReg>(sq->H, n, a, bad, sq->hscale);
    const int r = threadIdx.x;
#pragma unroll
    for (int c = 0; c < kCholReg; ++c)
        if (r < n && c <= r) sq->L[r * K + c] = a[c];
    if (r == 0) {
        sq->chol_bad = bad;
        sq->L_ver = hv;
    }
}

// Symmetric eigen-decomposition of A (n x n) by cyclic Jacobi with
// round-robin pairing (n/2 independent rotations per round), starting from
// the orthogonal V given; A ends diagonal, the columns of V are eigenvectors.
// A is a Gram matrix (positive semidefinite) formed in FP64, so its entries
// carry absolute errors of order eps trace(A): an entry is annihilated only
// while |a_pq| > 1e-14 sqrt(a_pp a_qq) + 1e-15 trace(A), and the sweeps end
// with the first one that rotates nothing (a test on the whole off-diagonal
// mass against 1e-30 of the diagonal's rarely passed once rounding noise
// dominated it, so most calls ran the sweep limit; a purely relative
// threshold never passes on such a matrix).  A round applies its rotations
// from both sides in one pass, J^T A J element by element (the column
// rotation first, then the row rotation, as two passes would), from A into
// the scratch B and back on the next round, with V J in the same pass: one
// barrier after the rotation angles, one after the update, none for a round
// that rotates nothing.  B is scratch of the same shape as A.
__device__ void jacobi_eig(double *A, double *B, double *V, int n)
{
    __shared__ double cs[K][2];          // rotation of the pair that index i belongs to
    __shared__ int mate[K], role[K];     // its partner and whether i is the pair's p (0) or q (1)
    __shared__ int s_rot, s_any[K];
    __shared__ double s_tr;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int m = (n + 1) & ~1;
    if (tid == 0) {
        double tr = 0.0;
        for (int i = 0; i < n; ++i) tr += fabs(A[i * K + i]);
        s_tr = tr;
    }
    __syncthreads();
    const double floor_abs = 1e-15 * s_tr;
    double *cur = A, *nxt = B;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) {
            s_rot = 0;
            for (int r = 0; r < m - 1; ++r) s_any[r] = 0;
        }
        __syncthreads();
        for (int round = 0; round < m - 1; ++round) {
            if (tid < m / 2) {
                auto slot = [&](int sl) { return sl == 0 ? 0 : 1 + (sl - 1 + round) % (m - 1); };
                int p = slot(tid), q = slot(m - 1 - tid);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, sn = 0.0;
                if (q < n) {
                    const double apq = cur[p * K + q];
                    const double thr =
                        1e-14 * sqrt(fabs(cur[p * K + p] * cur[q * K + q])) + floor_abs;
                    if (fabs(apq) > thr) {
                        s_rot = 1;
                        s_any[round] = 1;
                        const double th = (cur[q * K + q] - cur[p * K + p]) / (2.0 * apq);
                        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                    }
                    cs[p][0] = c; cs[p][1] = sn; mate[p] = q; role[p] = 0;
                    cs[q][0] = c; cs[q][1] = sn; mate[q] = p; role[q] = 1;
                } else if (p < n) {
                    cs[p][0] = 1.0; cs[p][1] = 0.0; mate[p] = p; role[p] = 0;
                }
            }
            __syncthreads();
            if (!s_any[round]) continue;          // uniform: nothing to rotate
            for (int t = tid; t < n * K; t += nt) {            // K: a constant divisor
                const int i = t / K, jj = t - i * K;
                if (jj >= n) continue;
                // column rotation of rows i and its mate at column jj, then the
                // row rotation of the pair of i
                const int pi = role[i] ? mate[i] : i, qi = role[i] ? i : mate[i];
                const int pj = role[jj] ? mate[jj] : jj, qj = role[jj] ? jj : mate[jj];
                const double cj = cs[jj][0], sj = cs[jj][1], ci = cs[i][0], si = cs[i][1];
                double col_p, col_q;       // (A J)[pi][jj], (A J)[qi][jj]
                if (pj == qj) {
                    col_p = cur[pi * K + jj];
                    col_q = cur[qi * K + jj];
                } else if (role[jj] == 0) {
                    col_p = cj * cur[pi * K + pj] - sj * cur[pi * K + qj];
                    col_q = cj * cur[qi * K + pj] - sj * cur[qi * K + qj];
                } else {
                    col_p = sj * cur[pi * K + pj] + cj * cur[pi * K + qj];
                    col_q = sj * cur[qi * K + pj] + cj * cur[qi * K + qj];
                }
                double v;
                if (pi == qi) v = col_p;
                else if (role[i] == 0) v = ci * col_p - si * col_q;
                else v = si * col_p + ci * col_q;
                nxt[i * K + jj] = v;
            }
            for (int t = tid; t < n * K; t += nt) {       // V <- V J (pairs of columns)
                const int r = t / K, jj = t - r * K;
                if (jj >= n || role[jj] != 0 || mate[jj] == jj) continue;
                const int q = mate[jj];
                const double c = cs[jj][0], sn = cs[jj][1];
                const double vp = V[r * K + jj], vq = V[r * K + q];
                V[r * K + jj] = c * vp - sn * vq;
                V[r * K + q] = sn * vp + c * vq;
            }
            __syncthreads();
            double *t2 = cur; cur = nxt; nxt = t2;
        }
        // every thread reads the flag before thread 0 clears it again
        const int rotated = s_rot;
        __syncthreads();
        if (!rotated) break;
    }
    if (cur != A) {
        for (int t = tid; t < n * n; t += nt) {
            const int i = t / n, jj = t - i * n;
            A[i * K + jj] = cur[i * K + jj];
        }
        __syncthreads();
    }
}

// The sequence state that the SPE start's dense step reads, requested by
// the whole block before the partial rows are reduced (one round trip
// alongside theirs instead of a chain of dependent loads): the column
// scales, the stored factor of H and whether it is current.
struct SpePre {
    double L[K * K];
    double s[K + 1];
    int use, bad;
};

// Range-checked raw buffer view of `bytes` bytes at p: a load at byte
// offset o reads memory only when 0 <= o < bytes and returns 0 otherwise,
// with no branch (so that the loads of one step go out together).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t seq_view(const void *p, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, bytes, 0x00020000);
}

__device__ __forceinline__ double view_f64(__amdgpu_buffer_rsrc_t r, int e)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8, 0, 0));
}

// The SPE start's inputs in registers of a 256-thread block: up to three
// factor entries and one scale per thread, the factor's currency words and
// the window size, all requested before any of them is used.
struct SpePreRegs {
    double l[(K * K + 255) / 256];
    double sc;
    int use, bad, k;
};

__device__ __forceinline__ void spe_pre_issue(const SeqDev *sq, SpePreRegs &r)
{
    const int tid = threadIdx.x;
    const __amdgpu_buffer_rsrc_t vl = seq_view(sq->L, K * K * 8), vs = seq_view(sq->s, (K + 1) * 8);
#pragma unroll
    for (int u = 0; u < (K * K + 255) / 256; ++u) r.l[u] = view_f64(vl, tid + 256 * u);
    r.sc = view_f64(vs, tid);
    r.use = sq->L_ver == sq->H_ver;
    r.bad = sq->chol_bad;
    r.k = sq->k;
}

__device__ __forceinline__ void spe_pre_commit(const SpePreRegs &r, SpePre *pre)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < (K * K + 255) / 256; ++u) {
        const int t = tid + 256 * u;
        if (t < K * K) pre->L[t] = r.l[u];
    }
    if (tid < K + 1) pre->s[tid] = r.sc;
    if (tid == 0) {
        pre->use = r.use;
        pre->bad = r.bad;
    }
}

// chol_solve_stored on the preloaded factor: the same substitutions on
// thread 0, in the same order, on the same values.
__device__ __forceinline__ bool chol_solve_pre(const SpePre *pre, double *y, const double *gv,
                                               int n, bool *good)
{
    if (!(n <= kCholReg && pre->use)) return false;
    if (threadIdx.x == 0) {
        const double *L = pre->L;
        for (int i = 0; i < n; ++i) {
            double t = gv[i];
            for (int j = 0; j < i; ++j) t -= L[i * K + j] * y[j];
            y[i] = t / L[i * K + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double t = y[i];
            for (int j = i + 1; j < n; ++j) t -= L[j * K + i] * y[j];
            y[i] = t / L[i * K + i];
        }
    }
    __syncthreads();
    *good = pre->bad == 0;
    return true;
}

// ------------------------------------------------------- dense steps
// val: the reduced values of the preceding basis product (see OP_* codes).
__device__ __forceinline__ void small_op(SeqDev *sq, int op, const double *val, double tol,
                                         ec_solve_info *info, const SpePre *pre = nullptr)
{
    __shared__ double Ms[K * K], Ls[K * K], Vs[K * K];
    __shared__ double ys[K + 1], gs[K + 1], sg[K + 1];
    __shared__ double cs2[2];
    __shared__ int ord[K];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int k = sq->k;
    switch (op) {
    case OP_SPE_START: {
        // g = q^T b, H y = g, x0 = q y, r0 = b - K q y
        const double *sc = pre ? pre->s : sq->s;
        for (int i = tid; i < k; i += nt) gs[i] = sc[i] * val[i];
        __syncthreads();
        bool good = k > 0;
        if (good && !(pre ? chol_solve_pre(pre, ys, gs, k, &good)
                          : chol_solve_stored(sq, Ls, ys, gs, k, &good)))
            good = chol_solve(sq->H, Ls, ys, gs, k, sq->hscale);
        // entries are independent: one per thread (no chain of dependent
        // global loads and stores on thread 0)
        for (int i = tid; i < K; i += nt) {
            const double c = (good && i < k) ? ys[i] * sc[i] : 0.0;
            sq->cA[i] = c;
            sq->cB[i] = -c;
        }
        if (tid == 0) {
            sq->flags = (k > 0 && !good) ? 1 : 0;
            sq->zero_start = good ? 0 : 1;
            sq->a1 = 0.0;
            sq->a2 = 1.0;
            sq->ncol_md = good ? k : 0;
            sq->active = 1;
            sq->push_on = 1;        // this solution is due for a push (see push_on)
        }
        break;
    }
    // PUSH1-3: the one-block form of the steps that push_coef and the slot
    // SpMV's acceptance test run in every block (batched pushes, where each
    // instance's grid is mostly small): the same expressions on the same
    // reduced values
    case OP_SPE_PUSH1: {
        // c1 = q^T x; w = x - q c1
        for (int i = tid; i < K; i += nt) {
            const double si = i < k ? sq->s[i] : 0.0;
            const double c1 = si * (i < k ? val[i] : 0.0);
            sq->c1[i] = c1;
            sq->cA[i] = -c1 * si;
        }
        if (tid == 0) {
            const double xx = val[k];
            sq->xnorm = sqrt(xx);
            sq->active = (sq->push_on && xx > 0.0 && xx <= 1e300) ? 1 : 0;
            sq->a1 = 1.0;
            sq->slot_new = k;
            sq->ncol_md = k;
            sq->accept = 0;     // set by the acceptance test for an accepted column
            sq->rotate = 0;     // set by OP_SPE_PUSH4 when the window slides
        }
        break;
    }
    case OP_SPE_PUSH2: {
        // second pass: c2 = q^T w; x2 = w - q c2
        for (int i = tid; i < K; i += nt) {
            const double si = i < k ? sq->s[i] : 0.0;
            const double c2 = si * (i < k ? val[i] : 0.0);
            sq->c2[i] = c2;
            sq->cA[i] = -c2 * si;
        }
        if (tid == 0) sq->a1 = 1.0;
        break;
    }
    case OP_SPE_PUSH3: {
        // accept x2 if it is not (numerically) in span(q): a linearly
        // independent new column
        if (tid == 0) {
            const double rho = sqrt(val[0]);
            sq->rho = rho;
            const int acc = (sq->active && rho > tol * sq->xnorm && k + 1 < K) ? 1 : 0;
            sq->accept = acc;
            sq->active = acc;
            if (acc) sq->s[k] = 1.0 / rho;
            sq->ncol_md = k + 1;
        }
        break;
    }
    case OP_SPE_PUSH4: {
        // new row/column of H = q^T K q and of the window coordinates R
        const int acc = sq->accept;
        if (acc) {
            const double sk = sq->s[k];
            for (int i = tid; i <= k; i += nt) {
                const double h = sq->s[i] * sk * val[i];
                sq->H[i * K + k] = h;
                sq->H[k * K + i] = h;
            }
            for (int i = tid; i < k; i += nt) {
                sq->R[i * K + k] = sq->c1[i] + sq->c2[i];
                sq->R[k * K + i] = 0.0;
            }
        }
        __syncthreads();
        if (tid == 0) {
            sq->rotate = 0;
            if (acc) {
                sq->R[k * K + k] = sq->rho;
                sq->k = k + 1;
                sq->w = sq->w + 1;
                sq->H_ver = sq->H_ver + 1;   // H grows (and may be downdated below)
            }
        }
        __syncthreads();
        if (!(sq->accept && sq->w > sq->cap)) break;
        // Drop the oldest solution: R' = R[:, 1:] (n x n-1) is upper
        // Hessenberg; Givens rotations Gt make Gt R' upper triangular with a
        // zero last row, so the window is spanned by the first n-1 columns of
        // q Gt^T; H' = Gt H Gt^T.
        const int n = sq->k;
        for (int t = tid; t < K * K; t += nt) {
            const int i = t / K, j = t - i * K;
            Ls[t] = (i < n && j < n - 1) ? sq->R[i * K + j + 1] : 0.0;
            Ms[t] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int j = 0; j < n - 1; ++j) {
            if (tid == 0) {
                const double a0 = Ls[j * K + j], b0 = Ls[(j + 1) * K + j];
                const double r = hypot(a0, b0);
                cs2[0] = r > 0.0 ? a0 / r : 1.0;
                cs2[1] = r > 0.0 ? b0 / r : 0.0;
            }
            __syncthreads();
            const double c = cs2[0], sn = cs2[1];
            for (int col = tid; col < n; col += nt) {
                if (col < n - 1) {
                    const double u = Ls[j * K + col], v = Ls[(j + 1) * K + col];
                    Ls[j * K + col] = c * u + sn * v;
                    Ls[(j + 1) * K + col] = -sn * u + c * v;
                }
                const double u = Ms[j * K + col], v = Ms[(j + 1) * K + col];
                Ms[j * K + col] = c * u + sn * v;
                Ms[(j + 1) * K + col] = -sn * u + c * v;
            }
            __syncthreads();
        }
        for (int t = tid; t < n * n; t += nt) {               // Vs = Gt H
            const int i = t / n, j = t - i * n;
            double s = 0.0;
            for (int l = 0; l < n; ++l) s += Ms[i * K + l] * sq->H[l * K + j];
            Vs[i * K + j] = s;
        }
        __syncthreads();
        for (int t = tid; t < K * K; t += nt) {
            const int i = t / K, j = t - i * K;
            double h = 0.0;
            if (i < n - 1 && j < n - 1)
                for (int l = 0; l < n; ++l) h += Vs[i * K + l] * Ms[j * K + l];
            sq->H[t] = h;
            sq->R[t] = (i < n - 1 && j < n - 1) ? Ls[t] : 0.0;
            // raw-column coefficients of the new basis: rot[i][j] = Gt[j][i] s_i
            sq->rot[t] = (i < n && j < n - 1) ? Ms[j * K + i] * sq->s[i] : 0.0;
        }
        __syncthreads();
        for (int i = tid; i <= K; i += nt) sq->s[i] = 1.0;
        if (tid == 0) {
            sq->rot_in = n;
            sq->rot_k = n - 1;
            sq->k = n - 1;
            sq->w = n - 1;
            sq->rotate = 1;
        }
        break;
    }
    case OP_POD_PUSH: {
        // new row/column of G = X^T X and H = X^T K X at the ring slot (a
        // push that is due: the push consumes the gate)
        if (tid == 0 && sq->push_on) {
            sq->push_on = 0;
            const int s = sq->slot_new, nc = sq->npush;
            for (int i = 0; i < nc; ++i) {
                sq->G[i * K + s] = val[2 * i];
                sq->G[s * K + i] = val[2 * i];
                sq->H[i * K + s] = val[2 * i + 1];
                sq->H[s * K + i] = val[2 * i + 1];
            }
            sq->count = nc;
            sq->head = (sq->head + 1) % sq->cap;
            sq->slot_new = sq->head;
            sq->npush = sq->count < sq->cap ? sq->count + 1 : sq->cap;
        }
        break;
    }
    case OP_POD_START: {
        const int n = sq->count;
        if (tid == 0) sq->push_on = 1;      // this solution is due for a push
        if (n == 0) {
            if (tid == 0) {
                sq->zero_start = 1; sq->kpod = 0; sq->pod_info = 1.0; sq->flags = 0;
                sq->a1 = 0.0; sq->a2 = 1.0; sq->ncol_md = 0; sq->active = 1;
                for (int i = 0; i < K; ++i) { sq->cA[i] = 0.0; sq->cB[i] = 0.0; }
            }
            break;
        }
        // warm start from the previous eigenvectors: A0 = V^T G V
        for (int t = tid; t < K * K; t += nt) Vs[t] = sq->V[t];
        __syncthreads();
        for (int t = tid; t < n * n; t += nt) {
            const int i = t / n, j = t - i * n;
            double s = 0.0;
            for (int l = 0; l < n; ++l) s += sq->G[i * K + l] * Vs[l * K + j];
            Ls[i * K + j] = s;
        }
        __syncthreads();
        for (int t = tid; t < n * n; t += nt) {
            const int i = t / n, j = t - i * n;
            double s = 0.0;
            for (int l = 0; l < n; ++l) s += Vs[l * K + i] * Ls[l * K + j];
            Ms[i * K + j] = s;
        }
        __syncthreads();
        jacobi_eig(Ms, Ls, Vs, n);
        // descending order of the eigenvalues (ties by index, a NaN below
        // every number, so that the ranks stay a permutation): thread i puts
        // i at its rank
        if (tid < n) {
            auto key = [](double v) { return v == v ? v : -INFINITY; };
            const double li = key(Ms[tid * K + tid]);
            int r = 0;
            for (int j = 0; j < n; ++j) {
                const double lj = key(Ms[j * K + j]);
                r += (lj > li || (lj == li && j < tid)) ? 1 : 0;
            }
            ord[r] = tid;
        }
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int i = 0; i < n; ++i) {
                const double l = Ms[ord[i] * K + ord[i]];
                sg[i] = l > 0.0 ? sqrt(l) : 0.0;
                tot += sg[i];
            }
            int kp = 0;
            for (int i = 0; i < n; ++i)
                if (sg[i] > 0.0 && sg[i] >= sq->pod_eps * sg[0]) ++kp;
            if (kp > sq->pod_kmax) kp = sq->pod_kmax;
            double kept = 0.0;
            for (int i = 0; i < kp; ++i) kept += sg[i];
            sq->kpod = kp;
            sq->pod_info = tot > 0.0 ? kept / tot : 1.0;
            for (int i = 0; i < n; ++i) sq->lam[i] = sg[i];
        }
        __syncthreads();
        for (int t = tid; t < K * K; t += nt) {                // sorted eigenvectors
            const int i = t / K, j = t - i * K;
            sq->V[t] = (i < n && j < n) ? Vs[i * K + ord[j]] : (i == j ? 1.0 : 0.0);
        }
        __syncthreads();
        // the sorted eigenvectors are Vs[., ord[.]] (the copy in sq->V above
        // is for the next call's warm start)
        const int kp = sq->kpod;
        for (int t = tid; t < n * kp; t += nt) {               // Ls = H V_k
            const int l = t / kp, b2 = t - l * kp;
            const int ob = ord[b2];
            double h = 0.0;
            for (int m2 = 0; m2 < n; ++m2) h += sq->H[l * K + m2] * Vs[m2 * K + ob];
            Ls[l * K + b2] = h;
        }
        __syncthreads();
        for (int t = tid; t < kp * kp; t += nt) {              // Sigma^-1 V_k^T H V_k Sigma^-1
            const int a2 = t / kp, b2 = t - a2 * kp;
            const int oa = ord[a2];
            double h = 0.0;
            for (int l = 0; l < n; ++l) h += Vs[l * K + oa] * Ls[l * K + b2];
            Ms[a2 * K + b2] = h / (sg[a2] * sg[b2]);
        }
        for (int a2 = tid; a2 < kp; a2 += nt) {                // Sigma^-1 V_k^T X^T b
            const int oa = ord[a2];
            double s = 0.0;
            for (int l = 0; l < n; ++l) s += Vs[l * K + oa] * val[l];
            gs[a2] = s / sg[a2];
        }
        __syncthreads();
        bool good = kp > 0;
        if (good) good = chol_solve(Ms, Ls, ys, gs, kp, sq->hscale);
        if (tid == 0) {
            // z = V_k Sigma_k^-1 y ; x0 = X z ; r0 = b - (K X) z
            for (int l = 0; l < K; ++l) {
                double z = 0.0;
                if (good && l < n)
                    for (int j = 0; j < kp; ++j) z += Vs[l * K + ord[j]] * ys[j] / sg[j];
                sq->cA[l] = z;
                sq->cB[l] = -z;
            }
            sq->flags = (kp > 0 && !good) ? 1 : 0;
            sq->zero_start = good ? 0 : 1;
            sq->a1 = 0.0;
            sq->a2 = 1.0;
            sq->ncol_md = good ? n : 0;
            sq->active = 1;
        }
        break;
    }
    default:
        break;
    }
    if (info && tid == 0 && (op == OP_SPE_START || op == OP_POD_START)) {
        info->basis_cols = op == OP_POD_START ? sq->kpod : sq->k;
        info->pod_info = op == OP_POD_START ? sq->pod_info : 1.0;
    }
    __syncthreads();
}

// -------------------------------------------------------- basis products
// part[(i*nb + j) * kMdBlocks + block] = sum over the block's rows of A_i B_j for p = k (+1 with
// a_extra) columns of A and nb <= 4 vectors B.  One wave handles 16 rows per
// step: lane (m = lane % 16, kq = lane / 16) loads 4 consecutive rows of A
// column m (and of B_m), so each 16-lane group reads full 128-byte lines;
// the four rows feed four v_mfma_f64_16x16x4f64 (K index kq = group), i.e.
// C[m][j] += A_m[row] B_j[row].
__device__ __forceinline__ void load4(const double *col, int64_t row, int64_t n, double (&v)[4])
{
    if (!col) {
        v[0] = v[1] = v[2] = v[3] = 0.0;
        return;
    }
    if (row + 3 < n) {
        const double2 *p = reinterpret_cast<const double2 *>(col + row);
        const double2 u0 = p[0], u1 = p[1];
        v[0] = u0.x; v[1] = u0.y; v[2] = u1.x; v[3] = u1.y;
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = (row + s < n) ? col[row + s] : 0.0;
    }
}

// The kernels below come in two launches: argument sets a0 / a1 by value
// (block row blockIdx.y picks one) or row blockIdx.y of a device table
// (independent sequences or instances in one launch); each set sees exactly
// the single-set grid.
__device__ __forceinline__ void multidot_body(const MdArgs &a)
{
    if (a.active && !*a.active) return;
    __shared__ double red[kMdWaves][32][4];
    const int k = a.kp ? *a.kp : a.kfix;
    const int p = k + (a.a_extra ? 1 : 0);
    const int nb = a.nb;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    auto colA = [&](int c) -> const double * {
        if (c >= p) return nullptr;
        return c < k ? a.A + (int64_t)c * a.ld : a.a_extra;
    };
    const double *cA0 = colA(m), *cA1 = colA(16 + m);
    const double *cB = nullptr;
    double bs = 1.0;
    switch (m) {
    case 0: if (nb > 0) { cB = a.B[0].p; bs = a.B[0].scale ? *a.B[0].scale : 1.0; } break;
    case 1: if (nb > 1) { cB = a.B[1].p; bs = a.B[1].scale ? *a.B[1].scale : 1.0; } break;
    case 2: if (nb > 2) { cB = a.B[2].p; bs = a.B[2].scale ? *a.B[2].scale : 1.0; } break;
    case 3: if (nb > 3) { cB = a.B[3].p; bs = a.B[3].scale ? *a.B[3].scale : 1.0; } break;
    default: break;
    }
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const int64_t n = a.n;
    const int64_t gw = (int64_t)blockIdx.x * kMdWaves + wv, nw = (int64_t)gridDim.x * kMdWaves;
    // two 16-row groups per iteration: every load of both groups is issued
    // before the matrix-core work that consumes them
    for (int64_t r0 = gw * 16; r0 < n; r0 += 2 * nw * 16) {
        const int64_t rowa = r0 + kq * 4, rowb = r0 + nw * 16 + kq * 4;
        double aa[4], ab[4], ba[4], bb[4];
        load4(cA0, rowa, n, aa);
        load4(cB, rowa, n, ba);
        load4(cA0, rowb, n, ab);
        load4(cB, rowb, n, bb);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            ba[s] *= bs;
            bb[s] *= bs;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[s], ba[s], acc0, 0, 0, 0);
#pragma unroll
        for (int s = 0; s < 4; ++s)
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ab[s], bb[s], acc0, 0, 0, 0);
        if (p > 16) {
            double a1[4], a2[4];
            load4(cA1, rowa, n, a1);
            load4(cA1, rowb, n, a2);
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], ba[s], acc1, 0, 0, 0);
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[s], bb[s], acc1, 0, 0, 0);
        }
    }
    // D layout (gfx950): lane l, element s holds C[4*s + l/16][l % 16]
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int row = 4 * s + kq;
        if (m < 4) {
            red[wv][row][m] = acc0[s];
            red[wv][16 + row][m] = acc1[s];
        }
    }
    __syncthreads();
    // one thread per value sums the waves in a fixed order
    const int nvals = p * nb;
    for (int t = threadIdx.x; t < nvals; t += blockDim.x) {
        const int i = t / nb, j = t - i * nb;
        double s = red[0][i][j];
#pragma unroll
        for (int w = 1; w < kMdWaves; ++w) s += red[w][i][j];
        a.part[(int64_t)t * kMdBlocks + blockIdx.x] = s;         // value-major
    }
}

__global__ void __launch_bounds__(kMdThreads) k_multidot(MdArgs a0, MdArgs a1)
{
    const MdArgs a = blockIdx.y ? a1 : a0;
    multidot_body(a);
}

__global__ void __launch_bounds__(kMdThreads) k_multidot_tab(const MdArgs *tab)
{
    multidot_body(tab[blockIdx.y]);
}

void multidot(const MdArgs &a, hipStream_t st, const MdArgs *a1)
{
    hipLaunchKernelGGL(k_multidot, dim3(kMdBlocks, a1 ? 2 : 1), dim3(kMdThreads), 0, st, a,
                       a1 ? *a1 : a);
}

void multidot_tab(const MdArgs *tab, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_multidot_tab, dim3(kMdBlocks, n), dim3(kMdThreads), 0, st, tab);
}

// ----------------------------------------------------- linear combinations
// y1 = a1 v1 + sum_{i<k} cA_i A_i        (y1 may be column *slot of A)
// y2 = a2 s2 v2 + sum_{i<k} cB_i B_i
// partials: [0..k) A_i^T y1 (want_dots), then |y1|^2, |y2|^2, |s2 v2|^2
// DOTS = a.want_dots, chosen on the host: the kernel without the dots does
// not carry their registers.
// The dense step OP_SPE_PUSH1 (c1 = q^T x, w = x - q c1, gate: a push that
// is due and a finite nonzero x) or OP_SPE_PUSH2 (c2 = q^T w, x2 = w - q c2)
// run by every block of the combination that applies it, on the reduced
// partials of the preceding product: the block's coefficients into sA, the
// gate into *gate, k into *kout.  Block 0 stores what the step stores; the
// other blocks read only fields that no block of this launch writes.
__device__ __forceinline__ void push_coef(SeqDev *sq, int op, const double *pin, double *sA,
                                          int *gate, int *kout)
{
    __shared__ double val[kMaxWin];
    const int k = sq->k;
    int nv = op == OP_SPE_PUSH1 ? k + 1 : sq->ncol_md + 3;
    nv = nv < 0 ? 0 : (nv > kMaxWin ? kMaxWin : nv);
    reduce_rows<kMaxWin>(pin, kMaxWin, nv, val);
    const bool b0 = blockIdx.x == 0;
    if (threadIdx.x < K) {
        const int i = threadIdx.x;
        const double si = i < k ? sq->s[i] : 0.0;
        const double c = si * (i < k ? val[i] : 0.0);
        sA[i] = i < k ? -c * si : 0.0;
        if (b0) {
            (op == OP_SPE_PUSH1 ? sq->c1 : sq->c2)[i] = c;
            sq->cA[i] = -c * si;
        }
    }
    if (threadIdx.x == 0) {
        int g;
        if (op == OP_SPE_PUSH1) {
            const double xx = val[k];
            g = (sq->push_on && xx > 0.0 && xx <= 1e300) ? 1 : 0;
            if (b0) {
                sq->xnorm = sqrt(xx);
                sq->active = g;
                sq->a1 = 1.0;
                sq->slot_new = k;
                sq->ncol_md = k;
                sq->accept = 0;     // set by the acceptance test for an accepted column
                sq->rotate = 0;     // set by OP_SPE_PUSH4 when the window slides
            }
        } else {
            g = sq->active;
            if (b0) sq->a1 = 1.0;
        }
        *gate = g;
        *kout = k;
    }
    __syncthreads();
}

// PRE: the kernel can run a dense step first (a.pre_seq); the table
// kernels of batched pushes never do, and leave that code out.
template <bool DOTS, bool PRE = true>
__device__ __forceinline__ void lincomb_body(const LcArgs &a)
{
    __shared__ double sA[kMaxWin], sB[kMaxWin];
    __shared__ double lds[kMaxWin + 3][kMdWaves];
    __shared__ int s_gate, s_k;
    int k;
    double a1;
    if (PRE && a.pre_seq) {
        if (threadIdx.x < kMaxWin) sB[threadIdx.x] = 0.0;
        push_coef(a.pre_seq, a.pre_op, a.pin, sA, &s_gate, &s_k);
        if (!s_gate) return;
        k = s_k;
        a1 = 1.0;
    } else {
        if (a.active && !*a.active) return;
        k = a.kp ? *a.kp : 0;
        if (threadIdx.x < kMaxWin) {
            sA[threadIdx.x] = (a.cA && (int)threadIdx.x < k) ? a.cA[threadIdx.x] : 0.0;
            sB[threadIdx.x] = (a.cB && (int)threadIdx.x < k) ? a.cB[threadIdx.x] : 0.0;
        }
        __syncthreads();
        a1 = a.a1 ? *a.a1 : 0.0;
    }
    double *y1 = a.y1;
    if (a.slot) y1 = const_cast<double *>(a.A) + (int64_t)(*a.slot) * a.ld;
    const double a2 = a.a2 ? *a.a2 : 0.0;
    const double s2 = a.v2.scale ? *a.v2.scale : 1.0;
    double dots[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) dots[i] = 0.0;
    double n1 = 0.0, n2 = 0.0, nbb = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < a.n; row += stride) {
        double v = (a.v1 && a1 != 0.0) ? a1 * a.v1[row] : 0.0;
        double u = 0.0;
#pragma unroll 4
        for (int i = 0; i < k; ++i) {
            v += sA[i] * a.A[(int64_t)i * a.ld + row];
            if (a.y2) u += sB[i] * a.B[(int64_t)i * a.ld + row];
        }
        if (y1) {
            y1[row] = v;
            n1 += v * v;
        }
        if (a.y2) {
            const double bv = a.v2.p ? s2 * a.v2.p[row] : 0.0;
            u += a2 * bv;
            a.y2[row] = u;
            n2 += u * u;
            nbb += bv * bv;
        }
        if constexpr (DOTS) {
            // second sweep over the same rows (cache hits): A_i^T y1 (holding
            // the row's entries in registers instead spilled and was slower)
#pragma unroll
            for (int i = 0; i < KC; ++i)
                if (i < k) dots[i] += a.A[(int64_t)i * a.ld + row] * v;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nv = DOTS ? k : 0;
#pragma unroll
    for (int i = 0; i < KC; ++i) {
        if (i < nv) {
            const double s = wave_sum(dots[i]);
            if (lane == 0) lds[i][wv] = s;
        }
    }
    {
        const double s0 = wave_sum(n1), s1 = wave_sum(n2), s2w = wave_sum(nbb);
        if (lane == 0) {
            lds[kMaxWin][wv] = s0;
            lds[kMaxWin + 1][wv] = s1;
            lds[kMaxWin + 2][wv] = s2w;
        }
    }
    __syncthreads();
    // one thread per value sums the waves in a fixed order (value-major)
    for (int t = threadIdx.x; t < nv + 3; t += blockDim.x) {
        const int q = t < nv ? t : kMaxWin + (t - nv);
        double s = lds[q][0];
#pragma unroll
        for (int w = 1; w < kMdWaves; ++w) s += lds[q][w];
        a.part[(int64_t)t * kMdBlocks + blockIdx.x] = s;
    }
}

// the two argument sets as one array in the kernel arguments: block row y
// reads set y at a run-time offset (not both sets loaded and selected)
struct LcPair {
    LcArgs s[2];
};

template <bool DOTS>
__global__ void __launch_bounds__(kMdThreads) k_lincomb(LcPair sets)
{
    lincomb_body<DOTS>(sets.s[blockIdx.y]);
}

template <bool DOTS>
__global__ void __launch_bounds__(kMdThreads) k_lincomb_tab(const LcArgs *tab)
{
    lincomb_body<DOTS, false>(tab[blockIdx.y]);
}

// both sets (and every table row) have the same want_dots
void lincomb(const LcArgs &a, hipStream_t st, const LcArgs *a1)
{
    const LcPair sets{{a, a1 ? *a1 : a}};
    if (a.want_dots)
        hipLaunchKernelGGL(k_lincomb<true>, dim3(kMdBlocks, a1 ? 2 : 1), dim3(kMdThreads), 0, st,
                           sets);
    else
        hipLaunchKernelGGL(k_lincomb<false>, dim3(kMdBlocks, a1 ? 2 : 1), dim3(kMdThreads), 0, st,
                           sets);
}

void lincomb_tab(const LcArgs *tab, int n, bool dots, hipStream_t st)
{
    if (dots)
        hipLaunchKernelGGL(k_lincomb_tab<true>, dim3(kMdBlocks, n), dim3(kMdThreads), 0, st, tab);
    else
        hipLaunchKernelGGL(k_lincomb_tab<false>, dim3(kMdBlocks, n), dim3(kMdThreads), 0, st, tab);
}

// In-place rotation of the first rot_in columns of A (and B) into rot_k
// columns: A'_j = sum_i rot[i][j] A_i.  One sweep over the rows for both
// matrices: every row's inputs of A and B are loaded together and each
// coefficient read from shared memory serves both.
__device__ __forceinline__ void rotate_body(const RotArgs &r)
{
    double *A = r.A, *B = r.B;
    const int64_t ld = r.ld, n = r.n;
    SeqDev *seq = r.seq;
    // the last kernel of an SPE push.  Block 0: the pushed solution is no
    // longer due, and the new H is factored for the next start (beside the
    // rotation, which the other blocks do)
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) seq->push_on = 0;
        chol_store(seq);
        return;
    }
    if (!seq->rotate) return;
    __shared__ double R[K * K];
    const int kin = seq->rot_in, kout = seq->rot_k;
    for (int t = threadIdx.x; t < K * K; t += blockDim.x) R[t] = seq->rot[t];
    __syncthreads();
    const int64_t stride = (int64_t)(gridDim.x - 1) * blockDim.x;
    for (int64_t row = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x; row < n;
         row += stride) {
        double va[KC], vb[KC];
#pragma unroll
        for (int i = 0; i < KC; ++i) {
            va[i] = 0.0;
            vb[i] = 0.0;
            if (i < kin) {
                va[i] = A[(int64_t)i * ld + row];
                vb[i] = B[(int64_t)i * ld + row];
            }
        }
#pragma unroll 1
        for (int j = 0; j < kout; ++j) {
            double sa = 0.0, sb = 0.0;
#pragma unroll
            for (int i = 0; i < KC; ++i) {
                if (i < kin) {
                    const double c = R[i * K + j];
                    sa += c * va[i];
                    sb += c * vb[i];
                }
            }
            A[(int64_t)j * ld + row] = sa;
            B[(int64_t)j * ld + row] = sb;
        }
    }
}

__global__ void __launch_bounds__(kMdThreads) k_rotate(RotArgs r0, RotArgs r1)
{
    rotate_body(blockIdx.y ? r1 : r0);
}

__global__ void __launch_bounds__(kMdThreads) k_rotate_tab(const RotArgs *tab)
{
    rotate_body(tab[blockIdx.y]);
}

void rotate(const RotArgs &r, hipStream_t st, const RotArgs *r1)
{
    hipLaunchKernelGGL(k_rotate, dim3(kMdBlocks, r1 ? 2 : 1), dim3(kMdThreads), 0, st, r,
                       r1 ? *r1 : r);
}

void rotate_tab(const RotArgs *tab, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_rotate_tab, dim3(kMdBlocks, n), dim3(kMdThreads), 0, st, tab);
}

// One block per argument set (blockIdx.y): reduce the partial rows of the
// preceding basis product, then run the dense step `op` of the sequence.
// OP >= 0: the step is fixed at compile time (one kernel per step, each with
// the registers of its own step only: a kernel holding every step took all
// 256 registers and no longer fitted on a CU beside the push kernels of the
// other branch); OP < 0: sa.op.
template <int OP>
__device__ __forceinline__ void small_body(const SmallArgs &sa)
{
    // SPE steps read at most cap + 1 <= kMaxWin values
    constexpr int NV = (OP == OP_SPE_START || OP == OP_SPE_PUSH4) ? kMaxWin : kMdStride;
    SeqDev *sq = sa.seq;
    const int op = OP >= 0 ? OP : sa.op;
    const int nvals = sa.nvals < NV ? sa.nvals : NV;
    const double *part = sa.part;
    __shared__ double val[NV];
    // exactly the values the producing product kernel wrote (state before the op)
    int nv = nvals;
    switch (op) {
    case OP_SPE_START: nv = sq->k; break;                 // q^T b
    case OP_POD_START: nv = sq->count; break;             // X^T b
    case OP_SPE_PUSH1: nv = sq->k + 1; break;             // [q, x]^T x
    case OP_SPE_PUSH2: nv = sq->ncol_md + 3; break;       // q^T w and three norms
    case OP_SPE_PUSH3: nv = 3; break;                     // norms only
    case OP_SPE_PUSH4: nv = sq->ncol_md; break;           // q^T (K_n + eta D^T D) t
    case OP_POD_PUSH: nv = 2 * sq->npush; break;          // X^T [x, K x]
    default: break;
    }
    nv = nv < 0 ? 0 : (nv > nvals ? nvals : nv);
    if constexpr (OP == OP_SPE_START) {
        // reduce_rows with every load (the sequence state and all nvals
        // partial rows) issued before the first is used: the same wave
        // butterflies and the same four-wave sum, so the same values
        __shared__ SpePre pre;
        __shared__ double tmp[NV][4];
        SpePreRegs pr;
        spe_pre_issue(sq, pr);
        const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
        double rv[NV];
        const __amdgpu_buffer_rsrc_t vp = seq_view(part, part ? nvals * kMdBlocks * 8 : 0);
#pragma unroll
        for (int q = 0; q < NV; ++q) rv[q] = view_f64(vp, q * kMdBlocks + tid);
        const int kk = pr.k < 0 ? 0 : (pr.k > nvals ? nvals : pr.k);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            if (q < kk) {
                const double sm = wave_sum(rv[q]);
                if (lane == 0) tmp[q][wv] = sm;
            }
        }
        spe_pre_commit(pr, &pre);
        __syncthreads();
        if (tid < kk) val[tid] = ((tmp[tid][0] + tmp[tid][1]) + tmp[tid][2]) + tmp[tid][3];
        __syncthreads();
        small_op(sq, op, val, sa.tol, sa.info, &pre);
        return;
    }
    if (part) reduce_rows<NV>(part, nvals, nv, val);
    __syncthreads();
    small_op(sq, op, val, sa.tol, sa.info);
}

template <int OP>
__global__ void __launch_bounds__(256) k_small(SmallArgs s0, SmallArgs s1)
{
    small_body<OP>(blockIdx.y ? s1 : s0);
}

template <int OP>
__global__ void __launch_bounds__(256) k_small_tab(const SmallArgs *tab)
{
    small_body<OP>(tab[blockIdx.y]);
}

template <int OP>
static void small_launch(const SmallArgs &a, hipStream_t st, const SmallArgs *a1)
{
    hipLaunchKernelGGL(k_small<OP>, dim3(1, a1 ? 2 : 1), dim3(256), 0, st, a, a1 ? *a1 : a);
}

template <int OP>
static void small_tab_launch(const SmallArgs *tab, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_small_tab<OP>, dim3(1, n), dim3(256), 0, st, tab);
}

// both sets have the same op
void small(const SmallArgs &a, hipStream_t st, const SmallArgs *a1)
{
    switch (a.op) {
    case OP_SPE_START: small_launch<OP_SPE_START>(a, st, a1); break;
    case OP_SPE_PUSH4: small_launch<OP_SPE_PUSH4>(a, st, a1); break;
    case OP_POD_PUSH: small_launch<OP_POD_PUSH>(a, st, a1); break;
    case OP_POD_START: small_launch<OP_POD_START>(a, st, a1); break;
    default: small_launch<-1>(a, st, a1); break;
    }
}

// every row of the table has the step op
void small_tab(const SmallArgs *tab, int n, int op, hipStream_t st)
{
    switch (op) {
    case OP_SPE_START: small_tab_launch<OP_SPE_START>(tab, n, st); break;
    case OP_SPE_PUSH4: small_tab_launch<OP_SPE_PUSH4>(tab, n, st); break;
    case OP_POD_PUSH: small_tab_launch<OP_POD_PUSH>(tab, n, st); break;
    case OP_POD_START: small_tab_launch<OP_POD_START>(tab, n, st); break;
    default: small_tab_launch<-1>(tab, n, st); break;
    }
}

// -------------------------------------------------------- sequence state
__global__ void k_seq_reset(SeqDev *sq)
{
    for (int i = threadIdx.x; i < K * K; i += blockDim.x) {
        sq->H[i] = 0.0; sq->R[i] = 0.0; sq->G[i] = 0.0; sq->rot[i] = 0.0;
        sq->V[i] = (i % (K + 1)) == 0 ? 1.0 : 0.0;
    }
    if (threadIdx.x == 0) {
        sq->k = 0; sq->w = 0; sq->kpod = 0; sq->head = 0; sq->count = 0;
        sq->accept = 0; sq->rotate = 0; sq->active = 0; sq->flags = 0; sq->zero_start = 1;
        sq->ncol_md = 0; sq->npush = 1; sq->slot_new = 0; sq->pod_info = 1.0; sq->rot_in = 0;
        sq->rot_k = 0; sq->push_on = 0;
        sq->H_ver = 0; sq->L_ver = 0; sq->chol_bad = 0;
        for (int i = 0; i <= K; ++i) sq->s[i] = 1.0;
    }
}

void seq_reset(SeqDev *seq, hipStream_t st)
{
    hipLaunchKernelGGL(k_seq_reset, dim3(1), dim3(256), 0, st, seq);
}

__global__ void k_seq_config(SeqDev *sq, int method, int cap, int kmax, double eps,
                             double hscale)
{
    sq->hscale = hscale;
    sq->method = method;
    sq->cap = cap;
    sq->pod_kmax = kmax;
    sq->pod_eps = eps;
}

void seq_config(SeqDev *seq, int method, int cap, int kmax, double eps, double hscale,
                hipStream_t st)
{
    hipLaunchKernelGGL(k_seq_config, dim3(1), dim3(1), 0, st, seq, method, cap, kmax, eps,
                       hscale);
}

__global__ void k_seq_push_on(SeqDev *sq) { sq->push_on = 1; }

void seq_push_on(SeqDev *seq, hipStream_t st)
{
    hipLaunchKernelGGL(k_seq_push_on, dim3(1), dim3(1), 0, st, seq);
}

}  // namespace ec
