// ec_capi.cpp -- host side of the C-ABI declared in ec.h: problem assembly
// and validation, workspace layout, and the launch sequences of solves,
// start vectors and explicit Euler steps.  All arithmetic on edge arrays runs
// in the kernels of ec_kernels.hip; this file only builds tables and drives.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "ec.h"
#include "ec_internal.h"

using namespace ec;

namespace {

thread_local std::string g_create_error;

constexpr double kDepTol = 1e-10;   // SPE default: drop a solution whose new direction is below this
constexpr int64_t kAlign = 256;

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// A roctx range over one phase of host work (enqueue of a step, a solve's
// start vector, its PCG, the update, the pushes).  rocprofv3 --marker-trace
// records them nested, on the host clock; the kernels a range enqueues run
// later on the stream, so the kernel trace gives their GPU time.  Without a
// profiler attached a push/pop pair is a call through an empty dispatch
// table.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

}  // namespace

struct ec_problem {
    std::string err;
    Geo g{};
    Mats mats{};
    int64_t npad = 0, S = 0, ncell = 0;
    int nc = 0;
    int64_t nn = 0;
    std::vector<uint8_t> cls, cmat;
    std::vector<int> cslot;
    std::vector<double> minv, msig;
    std::vector<double> xs;
    int has_cond = 0;
    int bblo[3] = {0, 0, 0}, bbhi[3] = {-1, -1, -1};
    int band_lo[3] = {0, 0, 0}, band_hi[3] = {-1, -1, -1};
    int wf = 0;
    double amp = 0, freq = 0, tau = 1;
    int64_t ramp = 1;
    // bound state
    bool bound = false;
    hipStream_t st = nullptr;
    char *ws = nullptr;
    int64_t ws_bytes = 0;
    int cap = 0;
    int64_t ld = 0;
    // FP64 edge vectors: state, source, CG buffers, scratch
    double *xs_d = nullptr, *sj = nullptr, *sc = nullptr, *ac = nullptr, *bcpl = nullptr;
    double *rb[2] = {}, *wb[2] = {}, *sb[2] = {}, *pv = nullptr;
    double *w = nullptr, *t2 = nullptr, *t3 = nullptr, *t4 = nullptr;
    // scratch of a second history push running in the same launches
    double *w_b = nullptr, *t2_b = nullptr, *t3_b = nullptr, *t4_b = nullptr;
    // grad-div weight of the SPE projection: eta0 = half the mean diagonal of
    // K_n on edges off the conductor, scaled by the caller's factor
    double eta0 = 0.0, gauge_rel = 1.0;
    // largest eigenvalue of M_c^{-1} K_S from the last ec_cfl (0: none since
    // bind or the last material change); steps with dt above 2 / cfl_lam fail
    double cfl_lam = 0.0;
    // adaptive steps (ec_set_adaptive_dt): device estimate of |lambda|_max and
    // the safety factor of the halving rule; null: fixed steps
    const double *adapt_lam = nullptr;
    double adapt_safety = 0.5;
    double dep_tol = kDepTol;    // SPE linear-independence threshold (relative)
    double seq_eta[EC_NSEQ] = {};  // grad-div weight the stored SPE matrix was built with
    // per-sequence iteration budget of the solves being captured (0 = maxit)
    int graph_iters[EC_NSEQ] = {};
    // the adjoint workspace the last forward pass filled (checkpoints)
    const void *adj_ws = nullptr;
    int64_t adj_steps = 0;
    int adj_every = 0;
    double adj_dt = 0.0;
    // FP32 vectors of the refinement's inner solve
    float *frb[2] = {}, *fwb[2] = {}, *fsb[2] = {}, *fpv = nullptr, *fd = nullptr;
    double *hist[EC_NSEQ] = {};
    uint8_t *cls_d = nullptr, *cmat_d = nullptr;
    int *cslot_d = nullptr;
    double *minv_d = nullptr, *cvec_d = nullptr;
    // stability estimate: the power iterate (compact), the cell records of
    // the operator and the cell pass's partials
    double *cvec2_d = nullptr, *cellv_d = nullptr, *part_cell = nullptr;
    // consistent conductivity matrix (ELL over the compact conducting edges,
    // built on the host from the materials) and the solves with it
    std::vector<int> m_idx;
    std::vector<double> m_val, m_dinv;
    double m_hscale = 0.0;
    int mass_kind = EC_MASS_LUMPED, mass_method = EC_SV_SPE, mass_win = 8, mass_maxit = 200;
    double mass_rtol = 1e-10;
    int mass_hint = 16;
    int64_t ldc = 0;
    int *m_idx_d = nullptr;
    double *m_val_d = nullptr, *m_dinv_d = nullptr;
    double *m_g = nullptr, *m_y = nullptr, *m_p = nullptr, *m_rb[2] = {}, *m_wb[2] = {},
           *m_sb[2] = {}, *m_w = nullptr, *m_t2 = nullptr, *m_t4 = nullptr, *m_hist = nullptr;
    double *m_part = nullptr, *m_part_md = nullptr;
    CgCtl *m_ctl = nullptr;
    SeqDev *mseq_d = nullptr;
    // implicit Euler / Newton: padded Newton state and matrix-product vectors,
    // compact residual, start, correction and GMRES vectors, the Arnoldi
    // basis, the GMRES record and partial sums
    double *i_a = nullptr, *i_v = nullptr, *i_b = nullptr, *i_s = nullptr, *i_u = nullptr;
    double *i_aold = nullptr, *i_F = nullptr, *i_x = nullptr, *i_w = nullptr, *i_jv = nullptr,
           *i_t = nullptr, *i_V = nullptr, *i_part = nullptr, *i_pn = nullptr, *i_norm = nullptr;
    GmDev *gm_d = nullptr;
    Mats *mats_d = nullptr;
    SeqDev *seq_d = nullptr;
    Ctrl *ctrl_d = nullptr;
    CgCtl *cg_d = nullptr;
    double *part_cg = nullptr, *part_md = nullptr, *part_ref = nullptr, *part_md_b = nullptr;
    unsigned *bar = nullptr;     // grid-barrier counters of the PCG tail kernel
    int tail_blocks = 0;         // persistent tail grid, FP64 (0: no tail available)
    int tail_blocks_f = 0;       // the same for the FP32 inner solves
    // 2.5D PCG iteration (large grids): column width, planes per block, tile
    // counts and its grid; used while cg_blocks == grid25
    int t25 = 0, kb25 = 0, nti25 = 0, ntj25 = 0, ntk25 = 0, grid25 = 0, node_blocks = 0;
    int seq_method[EC_NSEQ], seq_win[EC_NSEQ], seq_kmax[EC_NSEQ];
    double seq_eps[EC_NSEQ];
    int hint[EC_NSEQ];
    int cg_blocks = 0, tiles = 0;
    // host polling of the CG done flag (eager mode)
    int *pin = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    // side stream of a captured step (the history pushes run on it) and the
    // events that order it against the problem's stream
    hipStream_t side = nullptr;
    hipEvent_t sev[4] = {nullptr, nullptr, nullptr, nullptr};
    // start method of captured steps that were launched since the last
    // flush: their last coupling solution may still be due for a push
    int pending_meth = -1;
    ~ec_problem()
    {
        if (pin) (void)hipHostFree(pin);
        for (hipEvent_t &e : ev)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t &e : sev)
            if (e) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
    }
};

// ---------------------------------------------------------------- errors
static int32_t fail(ec_problem *h, int32_t code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_create_error = buf;
    return code;
}

#define HIP_TRY(h, expr)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(h, EC_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

static int32_t launch_check(ec_problem *h, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(h, EC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return EC_OK;
}

static bool aligned(const void *p) { return p && ((uintptr_t)p % 16 == 0); }

// ------------------------------------------------------------- assembly
// Edge (c, i, j, k) of the padded layout
static inline int64_t slot(const ec_problem *h, int c, int i, int j, int k)
{
    return (int64_t)c * h->S + ((int64_t)k * (h->g.ny + 1) + j) * (h->g.nx + 1) + i;
}

// Consistent conductivity matrix of the lowest-order edge elements (the
// last paragraph of Sec. III: a non-diagonal M_c).  In a conducting cell of
// sides h and conductivity sigma, the four edges of direction c couple with
// sigma h_a1 h_a2 / h_c times the integrals of products of the bilinear hats
// of the transverse face: 1/9 (the edge itself), 1/18 (a side apart), 1/36
// (diagonal); row sums are the lumped FIT M_sigma.  Rows over the compact
// conducting-edge list, at most kMassNnz entries each, ELL layout.
static void mass_build(ec_problem *h)
{
    const int nc = h->nc;
    const int px = h->g.px, py = h->g.py;
    const int64_t S = h->S;
    std::vector<int> pos(h->npad, -1);
    for (int t = 0; t < nc; ++t) pos[h->cslot[t]] = t;
    std::vector<int> cols((size_t)nc * kMassNnz, -1), cnt(nc, 0);
    std::vector<double> vals((size_t)nc * kMassNnz, 0.0);
    const double hh[3] = {h->g.hx, h->g.hy, h->g.hz};
    const double w4[4] = {1.0 / 9.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0};
    const int nx = h->g.nx, ny = h->g.ny, nz = h->g.nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int m = h->cmat[((int64_t)k * ny + j) * nx + i];
                if (!m) continue;
                const double sig = h->mats.sig[m];
                for (int c = 0; c < 3; ++c) {
                    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
                    const double scale = sig * hh[a1] * hh[a2] / hh[c];
                    int e4[4];
                    for (int q = 0; q < 4; ++q) {
                        int nd[3] = {i, j, k};
                        nd[a1] += q & 1;
                        nd[a2] += q >> 1;
                        e4[q] = pos[c * S + ((int64_t)nd[2] * py + nd[1]) * px + nd[0]];
                    }
                    for (int e = 0; e < 4; ++e)
                        for (int f = 0; f < 4; ++f) {
                            const int row = e4[e], col = e4[f];
                            if (row < 0 || col < 0) continue;
                            const double v = scale * w4[((e ^ f) & 1) + 2 * (((e ^ f) >> 1) & 1)];
                            int q = 0;
                            while (q < cnt[row] && cols[(size_t)row * kMassNnz + q] != col) ++q;
                            if (q == cnt[row]) {
                                cols[(size_t)row * kMassNnz + q] = col;
                                ++cnt[row];
                            }
                            vals[(size_t)row * kMassNnz + q] += v;
                        }
                }
            }
    h->m_idx.assign((size_t)std::max(nc, 1) * kMassNnz, -1);
    h->m_val.assign((size_t)std::max(nc, 1) * kMassNnz, 0.0);
    h->m_dinv.assign(std::max(nc, 1), 0.0);
    h->m_hscale = 0.0;
    for (int e = 0; e < nc; ++e)
        for (int q = 0; q < cnt[e]; ++q) {
            const int col = cols[(size_t)e * kMassNnz + q];
            const double v = vals[(size_t)e * kMassNnz + q];
            h->m_idx[(size_t)q * nc + e] = col;
            h->m_val[(size_t)q * nc + e] = v;
            if (col == e) {
                h->m_dinv[e] = 1.0 / v;
                h->m_hscale = std::max(h->m_hscale, v);
            }
        }
}

static int32_t assemble(ec_problem *h, const ec_grid *grid, const ec_materials *mat,
                        const ec_source *src)
{
    const int nx = grid->n[0], ny = grid->n[1], nz = grid->n[2];
    if (nx < 2 || ny < 2 || nz < 2 || nx > 1023 || ny > 1023 || nz > 1023)
        return fail(nullptr, EC_ERR_ARG, "grid: each axis needs 2..1023 cells");
    if (!(grid->len[0] > 0 && grid->len[1] > 0 && grid->len[2] > 0))
        return fail(nullptr, EC_ERR_ARG, "grid: lengths must be positive");
    const int64_t nodes = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    if (nodes >= (int64_t)1 << 25)
        return fail(nullptr, EC_ERR_ARG, "grid: at most 2^25 nodes");
    if (!mat || !mat->cell_mat || mat->n_mats < 0 || mat->n_mats >= kMaxMat ||
        (mat->n_mats > 0 && !mat->mats) || !(mat->nu0 > 0))
        return fail(nullptr, EC_ERR_ARG, "materials: bad descriptor (n_mats < %d, nu0 > 0)",
                    kMaxMat);
    Geo &g = h->g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.px = nx + 1; g.py = ny + 1;
    g.S = nodes;
    g.npad = 3 * nodes;
    g.hx = grid->len[0] / nx; g.hy = grid->len[1] / ny; g.hz = grid->len[2] / nz;
    h->S = nodes;
    h->npad = 3 * nodes;
    h->ncell = (int64_t)nx * ny * nz;
    Mats &M = h->mats;
    M.n = mat->n_mats + 1;
    M.nu0 = mat->nu0;
    M.sig[0] = 0.0; M.k1[0] = 0.0; M.k2[0] = 0.0; M.k3[0] = mat->nu0;
    for (int m = 0; m < mat->n_mats; ++m) {
        const ec_material &e = mat->mats[m];
        if (!(e.sigma > 0) || !std::isfinite(e.sigma) || !(e.k1 >= 0) || !std::isfinite(e.k2) ||
            !(e.k3 > 0) || !std::isfinite(e.k1) || !std::isfinite(e.k3))
            return fail(nullptr, EC_ERR_ARG,
                        "material %d: need sigma > 0, k1 >= 0, k3 > 0 and finite k2", m + 1);
        M.sig[m + 1] = e.sigma; M.k1[m + 1] = e.k1; M.k2[m + 1] = e.k2; M.k3[m + 1] = e.k3;
    }
    // Face weights of the nonconducting region: nu0 * dual edge / face area
    g.wx = mat->nu0 * g.hx / (g.hy * g.hz);
    g.wy = mat->nu0 * g.hy / (g.hz * g.hx);
    g.wz = mat->nu0 * g.hz / (g.hx * g.hy);
    // Jacobi: an edge off the conductor has four nonconducting faces
    g.dinv[0] = 1.0 / (2.0 * (g.wy + g.wz));
    g.dinv[1] = 1.0 / (2.0 * (g.wz + g.wx));
    g.dinv[2] = 1.0 / (2.0 * (g.wx + g.wy));
    h->eta0 = (1.0 / g.dinv[0] + 1.0 / g.dinv[1] + 1.0 / g.dinv[2]) / 6.0;

    h->cmat.assign(mat->cell_mat, mat->cell_mat + h->ncell);
    int lo[3] = {nx, ny, nz}, hi[3] = {-1, -1, -1};
    int64_t ncond = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int m = h->cmat[((int64_t)k * ny + j) * nx + i];
                if (m > mat->n_mats)
                    return fail(nullptr, EC_ERR_ARG, "cell_mat: id %d beyond n_mats", m);
                if (m) {
                    ++ncond;
                    lo[0] = std::min(lo[0], i); hi[0] = std::max(hi[0], i);
                    lo[1] = std::min(lo[1], j); hi[1] = std::max(hi[1], j);
                    lo[2] = std::min(lo[2], k); hi[2] = std::max(hi[2], k);
                }
            }
    h->has_cond = ncond > 0;
    for (int a = 0; a < 3; ++a) { h->bblo[a] = lo[a]; h->bbhi[a] = hi[a]; }
    const int64_t bvol = ncond ? (int64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1) : 0;
    g.box = (bvol == ncond) ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        g.clo[a] = ncond ? lo[a] : 1;
        g.chi[a] = ncond ? hi[a] : 0;
    }
    // Edge classes and M_sigma: sigma of the (up to four) cells around an
    // edge, a quarter of the dual face each, over the edge length.
    h->cls.assign(h->npad, 0);
    h->msig.assign(h->npad, 0.0);
    const int n3[3] = {nx, ny, nz};
    const double hh[3] = {g.hx, g.hy, g.hz};
    for (int c = 0; c < 3; ++c) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        const double quarter = hh[a1] * hh[a2] / 4.0 / hh[c];
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i <= nx; ++i) {
                    const int idx[3] = {i, j, k};
                    if (idx[c] >= n3[c]) continue;                           // padding
                    if (idx[a1] == 0 || idx[a1] == n3[a1] || idx[a2] == 0 || idx[a2] == n3[a2])
                        continue;                                            // Dirichlet
                    double s = 0.0;
                    for (int d1 = -1; d1 <= 0; ++d1)
                        for (int d2 = -1; d2 <= 0; ++d2) {
                            int cc[3] = {i, j, k};
                            cc[a1] += d1;
                            cc[a2] += d2;
                            s += M.sig[h->cmat[((int64_t)cc[2] * ny + cc[1]) * nx + cc[0]]];
                        }
                    const int64_t e = slot(h, c, i, j, k);
                    h->msig[e] = s * quarter;
                    h->cls[e] = s > 0.0 ? 1 : 2;
                }
    }
    h->cslot.clear();
    h->minv.clear();
    h->nn = 0;
    for (int64_t e = 0; e < h->npad; ++e) {
        if (h->cls[e] == 1) {
            h->cslot.push_back((int)e);
            h->minv.push_back(1.0 / h->msig[e]);
        } else if (h->cls[e] == 2) {
            ++h->nn;
        }
    }
    h->nc = (int)h->cslot.size();
    mass_build(h);
    // band of nonconducting edges coupled to the conductor (K_cn^T support)
    for (int a = 0; a < 3; ++a) {
        h->band_lo[a] = std::max(0, lo[a] - 1);
        h->band_hi[a] = std::min(n3[a], hi[a] + 2);
    }
    // Source
    if (!src || !src->edge_current)
        return fail(nullptr, EC_ERR_ARG, "source: edge_current is required");
    if (src->waveform < EC_WF_DC || src->waveform > EC_WF_EXP)
        return fail(nullptr, EC_ERR_ARG, "source: unknown waveform %d", src->waveform);
    if (src->waveform == EC_WF_RAMP && src->ramp_steps < 1)
        return fail(nullptr, EC_ERR_ARG, "source: ramp_steps must be >= 1");
    if (src->waveform == EC_WF_EXP && !(src->tau > 0))
        return fail(nullptr, EC_ERR_ARG, "source: tau must be positive");
    h->wf = src->waveform; h->amp = src->amp; h->freq = src->freq; h->tau = src->tau;
    h->ramp = src->ramp_steps;
    h->xs.assign(src->edge_current, src->edge_current + h->npad);
    double jmax = 0.0;
    for (int64_t e = 0; e < h->npad; ++e) {
        const double v = h->xs[e];
        if (!std::isfinite(v)) return fail(nullptr, EC_ERR_ARG, "source: non-finite entry");
        if (v != 0.0 && h->cls[e] != 2)
            return fail(nullptr, EC_ERR_ARG,
                        "source: X_S must vanish off the nonconducting edges (slot %lld)",
                        (long long)e);
        jmax = std::max(jmax, std::fabs(v));
    }
    // discrete divergence G^T X_S at every node
    double dmax = 0.0;
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double d = 0.0;
                if (i < nx) d -= h->xs[slot(h, 0, i, j, k)];
                if (i > 0) d += h->xs[slot(h, 0, i - 1, j, k)];
                if (j < ny) d -= h->xs[slot(h, 1, i, j, k)];
                if (j > 0) d += h->xs[slot(h, 1, i, j - 1, k)];
                if (k < nz) d -= h->xs[slot(h, 2, i, j, k)];
                if (k > 0) d += h->xs[slot(h, 2, i, j, k - 1)];
                dmax = std::max(dmax, std::fabs(d));
            }
    if (dmax > 1e-10 * jmax)
        return fail(nullptr, EC_ERR_ARG,
                    "source: X_S is not divergence free (|G^T X_S| = %g, |X_S| = %g)", dmax, jmax);
    return EC_OK;
}

extern "C" int32_t ec_create(const ec_grid *grid, const ec_materials *mat, const ec_source *src,
                             ec_handle *out)
{
    if (!out) return fail(nullptr, EC_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!grid) return fail(nullptr, EC_ERR_ARG, "grid is NULL");
    ec_problem *h = new (std::nothrow) ec_problem();
    if (!h) return fail(nullptr, EC_ERR_ARG, "out of host memory");
    int32_t st;
    try {
        st = assemble(h, grid, mat, src);
    } catch (...) {
        st = fail(nullptr, EC_ERR_ARG, "host allocation failed");
    }
    if (st != EC_OK) {
        delete h;
        return st;
    }
    for (int s = 0; s < EC_NSEQ; ++s) {
        h->seq_method[s] = -1; h->seq_win[s] = 0; h->seq_kmax[s] = 0; h->seq_eps[s] = 0.0;
    }
    *out = h;
    return EC_OK;
}

extern "C" int32_t ec_destroy(ec_handle h)
{
    if (!h) return EC_OK;
    // drain the problem's streams before their events, the side stream and
    // the pinned polling buffer go (work still queued may signal them)
    if (h->bound) {
        (void)hipStreamSynchronize(h->st);
        if (h->side) (void)hipStreamSynchronize(h->side);
    }
    delete h;
    return EC_OK;
}

// -------------------------------------------------------- workspace
// Layout (256-byte aligned pieces):
//   20 FP64 edge vectors, 8 FP32 edge vectors, per sequence 2 (cap+1) basis
//   columns, tables (classes, cell materials, conducting slots, 1/M_sigma),
//   sequence states, barrier, control block, reduction partials.
static int64_t layout(ec_problem *h, int cap, char *base)
{
    int64_t off = 0;
    auto take = [&](int64_t bytes) -> char * {
        const int64_t o = off;
        off = align_up(off + bytes, kAlign);
        return base ? base + o : nullptr;
    };
    const int64_t ld = align_up(h->npad, 64);
    double **vecs[] = {&h->xs_d, &h->sj, &h->sc, &h->ac, &h->bcpl, &h->rb[0], &h->rb[1],
                       &h->wb[0], &h->wb[1], &h->sb[0], &h->sb[1], &h->pv, &h->w, &h->t2,
                       &h->t3, &h->t4, &h->w_b, &h->t2_b, &h->t3_b, &h->t4_b};
    for (double **v : vecs) *v = (double *)take(ld * 8);
    float **fv[] = {&h->frb[0], &h->frb[1], &h->fwb[0], &h->fwb[1], &h->fsb[0], &h->fsb[1],
                    &h->fpv, &h->fd};
    for (float **v : fv) *v = (float *)take(ld * 4);
    for (int s = 0; s < EC_NSEQ; ++s) h->hist[s] = (double *)take(2 * (int64_t)(cap + 1) * ld * 8);
    h->cls_d = (uint8_t *)take(h->npad);
    h->cmat_d = (uint8_t *)take(h->ncell);
    h->cslot_d = (int *)take((int64_t)std::max(h->nc, 1) * 4);
    h->minv_d = (double *)take((int64_t)std::max(h->nc, 1) * 8);
    h->cvec_d = (double *)take((int64_t)std::max(h->nc, 1) * 8);
    h->cvec2_d = (double *)take((int64_t)std::max(h->nc, 1) * 8);
    h->cellv_d = (double *)take(std::max<int64_t>(h->ncell, 1) * kCellRec * 8);
    h->part_cell = (double *)take((h->ncell + 255) / 256 * 8 + 8);
    {
        const int64_t nc1 = std::max(h->nc, 1);
        const int64_t ldc = align_up(nc1, 64);
        h->m_idx_d = (int *)take(kMassNnz * nc1 * 4);
        h->m_val_d = (double *)take(kMassNnz * nc1 * 8);
        h->m_dinv_d = (double *)take(nc1 * 8);
        double **mv[] = {&h->m_g, &h->m_y, &h->m_p, &h->m_rb[0], &h->m_rb[1], &h->m_wb[0],
                         &h->m_wb[1], &h->m_sb[0], &h->m_sb[1], &h->m_w, &h->m_t2, &h->m_t4};
        for (double **v : mv) *v = (double *)take(ldc * 8);
        h->m_hist = (double *)take(2 * (int64_t)(cap + 1) * ldc * 8);
        h->m_part = (double *)take(2 * 4 * (int64_t)kMaxBlocks * 8);
        h->m_part_md = (double *)take((int64_t)kMdBlocks * kMdStride * 8);
        h->m_ctl = (CgCtl *)take(2 * sizeof(CgCtl));
        h->mseq_d = (SeqDev *)take(sizeof(SeqDev));
        h->ldc = ldc;
        double **ip[] = {&h->i_a, &h->i_v, &h->i_b, &h->i_s, &h->i_u};
        for (double **v : ip) *v = (double *)take(ld * 8);
        double **ic[] = {&h->i_aold, &h->i_F, &h->i_x, &h->i_w, &h->i_jv, &h->i_t};
        for (double **v : ic) *v = (double *)take(ldc * 8);
        h->i_V = (double *)take((int64_t)(kGmMax + 1) * ldc * 8);
        h->i_part = (double *)take((int64_t)kMdBlocks * kMdStride * 8);
        h->i_pn = (double *)take(256 * 8);
        h->i_norm = (double *)take(8 * 8);
        h->gm_d = (GmDev *)take(sizeof(GmDev));
    }
    h->mats_d = (Mats *)take(sizeof(Mats));
    h->seq_d = (SeqDev *)take(sizeof(SeqDev) * EC_NSEQ);
    h->ctrl_d = (Ctrl *)take(sizeof(Ctrl));
    h->cg_d = (CgCtl *)take(2 * sizeof(CgCtl));
    h->part_cg = (double *)take(2 * 4 * (int64_t)kMaxBlocks * 8);
    h->part_md = (double *)take((int64_t)kMdBlocks * kMdStride * 8);
    h->part_md_b = (double *)take((int64_t)kMdBlocks * kMdStride * 8);
    h->part_ref = (double *)take(2 * (int64_t)kMaxBlocks * 8);
    h->bar = (unsigned *)take((int64_t)kBarWords * kBarStride * sizeof(unsigned));
    h->ld = ld;
    return off;
}

extern "C" int32_t ec_sizes(ec_handle h, int32_t window_cap, int64_t *n_padded, int64_t *n_c,
                            int64_t *n_n, int64_t *workspace_bytes)
{
    if (!h) return fail(nullptr, EC_ERR_ARG, "handle is NULL");
    if (window_cap < 1 || window_cap > EC_MAX_WINDOW)
        return fail(h, EC_ERR_ARG, "window_cap must be 1..%d", EC_MAX_WINDOW);
    if (n_padded) *n_padded = h->npad;
    if (n_c) *n_c = h->nc;
    if (n_n) *n_n = h->nn;
    if (workspace_bytes) {
        ec_problem tmp;   // layout on a scratch copy: do not disturb bound pointers
        tmp.npad = h->npad; tmp.S = h->S; tmp.ncell = h->ncell; tmp.nc = h->nc;
        *workspace_bytes = layout(&tmp, window_cap, nullptr);
    }
    return EC_OK;
}

// Grid of the node kernels: one tile of 256 nodes per block up to kMaxBlocks
// (then a block sweeps several tiles); a multiple of 8 for the XCD mapping.
// Shape of the 2.5D iteration.  Column width TI (x 256/TI nodes): least
// idle threads, the widest on ties (contiguous rows along i beat a smaller
// halo: 128^3 measured 151 us at 64x4 vs 168 us at 16x16); then the fewest
// planes per block (>= 16: the march fetches each plane one plane ahead, so
// longer columns amortise its start; 128^3: 111 us at 16 planes) that keep
// the grid within kMaxBlocks.
// ti / kb > 0 force a shape.  Returns false when it does not fit (or, without
// force, when the grid is too small to fill the chip with it).
static bool plan_25(ec_problem *h, bool force, int ti_want = 0, int kb_want = 0)
{
    const int nx = h->g.nx, ny = h->g.ny, nz = h->g.nz;
    if (!force && (int64_t)nx * ny * nz < (int64_t)96 * 96 * 96) return false;
    double best = 1e300;
    int bt = 0;
    for (int ti : {64, 32, 16}) {
        if (ti_want && ti != ti_want) continue;
        const int tj = 256 / ti;
        const int64_t cover = (int64_t)((nx + ti - 1) / ti) * ti * (((ny + tj - 1) / tj) * tj);
        const double waste = (double)cover / ((double)nx * ny);
        if (waste < best - 1e-9) {
            best = waste;
            bt = ti;
        }
    }
    if (!bt) return false;
    const int tj = 256 / bt, nti = (nx + bt - 1) / bt, ntj = (ny + tj - 1) / tj;
    int kb = kb_want > 0 ? std::min(kb_want, nz) : std::min(16, nz), ntk = 0;
    for (;; kb = std::min(nz, kb * 2)) {
        ntk = (nz + kb - 1) / kb;
        if (align_up((int64_t)nti * ntj * ntk, 8) <= kMaxBlocks || kb >= nz || kb_want > 0) break;
    }
    const int64_t grid = align_up((int64_t)nti * ntj * ntk, 8);
    if (grid > kMaxBlocks) return false;
    h->t25 = bt; h->kb25 = kb; h->nti25 = nti; h->ntj25 = ntj; h->ntk25 = ntk;
    h->grid25 = (int)grid;
    return true;
}

static int choose_blocks(ec_problem *h)
{
    const int64_t tiles = (h->S + kTile - 1) / kTile;
    const int64_t b = std::min<int64_t>(align_up(tiles, 8), kMaxBlocks);
    return (int)std::max<int64_t>(b, 8);
}

// consistent M_c table to the device (bound handles)
static int32_t mass_upload(ec_problem *h)
{
    if (!h->nc) return EC_OK;
    const size_t n9 = (size_t)h->nc * kMassNnz;
    HIP_TRY(h, hipMemcpyAsync(h->m_idx_d, h->m_idx.data(), n9 * 4, hipMemcpyHostToDevice, h->st));
    HIP_TRY(h, hipMemcpyAsync(h->m_val_d, h->m_val.data(), n9 * 8, hipMemcpyHostToDevice, h->st));
    HIP_TRY(h, hipMemcpyAsync(h->m_dinv_d, h->m_dinv.data(), (size_t)h->nc * 8,
                              hipMemcpyHostToDevice, h->st));
    return EC_OK;
}

// largest diagonal entry of K_n (the Jacobi diagonal of the x, y, z edges)
static double kn_diag_max(const ec_problem *h)
{
    return 1.0 / std::min(h->g.dinv[0], std::min(h->g.dinv[1], h->g.dinv[2]));
}

// The first dispatch of a kernel with a private segment on a hardware queue
// makes the runtime set up that queue's scratch, with the queue idle for
// about 0.13 ms (twice when a larger segment follows).  The branches of a
// captured step run on queues the library's streams need not have used
// eagerly, so the first replay of the first captured step of a process paid
// it (the PCG iteration and the SPE start's dense step have small private
// segments, from spill frames).  Once per device, a
// dispatch with a larger segment than any library kernel on a fresh stream
// per hardware queue (HIP assigns streams to its GPU_MAX_HW_QUEUES queues in
// turn, 4 by default) sets every queue up at bind.
static int32_t warm_queue_scratch(ec_problem *h)
{
    static bool warmed[64] = {};
    int dev = 0;
    HIP_TRY(h, hipGetDevice(&dev));
    if (dev < 0 || dev >= 64 || warmed[dev]) return EC_OK;
    int nq = 4;
    if (const char *e = std::getenv("GPU_MAX_HW_QUEUES")) nq = std::atoi(e);
    nq = std::min(std::max(nq, 1), 32);
    std::vector<hipStream_t> ss(nq, nullptr);
    hipError_t e = hipSuccess;
    for (int q = 0; q < nq && e == hipSuccess; ++q) {
        e = hipStreamCreateWithFlags(&ss[q], hipStreamNonBlocking);
        if (e == hipSuccess) {
            scratch_warm(ss[q]);
            e = hipGetLastError();
        }
    }
    for (hipStream_t s : ss) {
        if (!s) continue;
        hipError_t e2 = hipStreamSynchronize(s);
        if (e == hipSuccess) e = e2;
        (void)hipStreamDestroy(s);
    }
    if (e != hipSuccess) return fail(h, EC_ERR_HIP, "queue scratch set-up: %s", hipGetErrorString(e));
    warmed[dev] = true;
    return EC_OK;
}

extern "C" int32_t ec_bind(ec_handle h, void *hip_stream, void *workspace, int64_t bytes,
                           int32_t window_cap)
{
    if (!h) return fail(nullptr, EC_ERR_ARG, "handle is NULL");
    if (window_cap < 1 || window_cap > EC_MAX_WINDOW)
        return fail(h, EC_ERR_ARG, "window_cap must be 1..%d", EC_MAX_WINDOW);
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0)
        return fail(h, EC_ERR_ARG, "workspace must be non-NULL and 256-byte aligned");
    {
        ec_problem tmp;
        tmp.npad = h->npad; tmp.S = h->S; tmp.ncell = h->ncell; tmp.nc = h->nc;
        const int64_t need = layout(&tmp, window_cap, nullptr);
        if (bytes < need)
            return fail(h, EC_ERR_ARG, "workspace too small: %lld < %lld bytes", (long long)bytes,
                        (long long)need);
    }
    h->st = (hipStream_t)hip_stream;
    h->ws = (char *)workspace;
    h->ws_bytes = bytes;
    h->cap = window_cap;
    layout(h, window_cap, h->ws);
    h->g.cls = h->cls_d;
    hipStream_t st = h->st;
    HIP_TRY(h, hipMemsetAsync(h->ws, 0, (size_t)bytes, st));
    HIP_TRY(h, hipMemcpyAsync(h->xs_d, h->xs.data(), h->npad * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->cls_d, h->cls.data(), h->npad, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->cmat_d, h->cmat.data(), h->ncell, hipMemcpyHostToDevice, st));
    if (h->nc) {
        HIP_TRY(h, hipMemcpyAsync(h->cslot_d, h->cslot.data(), (size_t)h->nc * 4,
                                  hipMemcpyHostToDevice, st));
        HIP_TRY(h, hipMemcpyAsync(h->minv_d, h->minv.data(), (size_t)h->nc * 8,
                                  hipMemcpyHostToDevice, st));
    }
    HIP_TRY(h, hipMemcpyAsync(h->mats_d, &h->mats, sizeof(Mats), hipMemcpyHostToDevice, st));
    {
        int32_t rc = mass_upload(h);
        if (rc) return rc;
        seq_config(h->mseq_d, EC_SV_SPE, window_cap, window_cap, 1e-4, h->m_hscale, st);
        seq_reset(h->mseq_d, st);
        h->mass_win = std::min(h->mass_win, window_cap);
    }
    Ctrl c{};
    c.one = 1.0;
    c.worst = EC_OK;
    HIP_TRY(h, hipMemcpyAsync(h->ctrl_d, &c, sizeof c, hipMemcpyHostToDevice, st));
    for (int s = 0; s < EC_NSEQ; ++s) {
        seq_config(h->seq_d + s, EC_SV_SPE, window_cap, window_cap, 1e-4, kn_diag_max(h), st);
        seq_reset(h->seq_d + s, st);
        h->seq_method[s] = -1;
        h->hint[s] = 16;
    }
    HIP_TRY(h, hipStreamSynchronize(st));
    if (!h->pin) HIP_TRY(h, hipHostMalloc((void **)&h->pin, 128, hipHostMallocDefault));
    for (hipEvent_t &e : h->ev)
        if (!e) HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (hipEvent_t &e : h->sev)
        if (!e) HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (!h->side) HIP_TRY(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    {
        int rc = warm_queue_scratch(h);
        if (rc) return rc;
    }
    h->pending_meth = -1;
    h->cfl_lam = 0.0;
    h->tiles = (int)((h->S + kTile - 1) / kTile);
    h->node_blocks = choose_blocks(h);
    h->cg_blocks = plan_25(h, false) ? h->grid25 : h->node_blocks;
    h->tail_blocks = cg_tail_blocks<double>();
    h->tail_blocks_f = cg_tail_blocks<float>();
    h->bound = true;
    return EC_OK;
}

#define NEED_BOUND(h)                                                                     \
    do {                                                                                  \
        if (!(h)) return fail(nullptr, EC_ERR_ARG, "handle is NULL");                     \
        if (!(h)->bound) return fail((h), EC_ERR_STATE, "ec_bind first");                 \
    } while (0)

// --------------------------------------------------------- histories
static double *basis_Q(ec_problem *h, int seq) { return h->hist[seq]; }
static double *basis_KQ(ec_problem *h, int seq)
{
    return h->hist[seq] + (int64_t)(h->cap + 1) * h->ld;
}

static void seq_ensure(ec_problem *h, int seq, int method, int window, int kmax, double eps)
{
    if (method != EC_SV_SPE && method != EC_SV_POD) return;
    if (h->seq_method[seq] == method && h->seq_win[seq] == window && h->seq_kmax[seq] == kmax &&
        h->seq_eps[seq] == eps)
        return;
    seq_config(h->seq_d + seq, method, window, kmax, eps, kn_diag_max(h), h->st);
    // the POD truncation parameters act on the next start vector only; a new
    // method or window starts a new history
    if (h->seq_method[seq] != method || h->seq_win[seq] != window) seq_reset(h->seq_d + seq, h->st);
    h->seq_method[seq] = method;
    h->seq_win[seq] = window;
    h->seq_kmax[seq] = kmax;
    h->seq_eps[seq] = eps;
}

// Grad-div weight of SPE pushes.  FP32-refined solves leave a gradient part
// of about (iterations x FP32 epsilon) in their solutions, far above FP64
// round-off; at the full weight the projection trades that invisible part for
// range error the residual sees (more so on finer grids, where the ratio of
// the largest to the smallest K_n eigenvalue grows), so those sequences use
// 1e-6 of it: enough to damp the growth of that part, too small to bias the
// projection.
constexpr double kRefinedGaugeScale = 1e-6;

static double spe_eta(const ec_problem *h, int precision)
{
    return h->gauge_rel * h->eta0 * (precision == EC_PREC_FP32_REFINED ? kRefinedGaugeScale : 1.0);
}

// an SPE history holds Q^T (K_n + eta D^T D) Q for one eta: a new weight
// starts a new history
static void seq_eta_ensure(ec_problem *h, int seq, int method, double eta)
{
    if (method != EC_SV_SPE || h->seq_eta[seq] == eta) return;
    seq_reset(h->seq_d + seq, h->st);
    h->seq_eta[seq] = eta;
}

static MdArgs md_args(ec_problem *h, double *part = nullptr)
{
    MdArgs m{};
    m.ld = h->ld;
    m.part = part ? part : h->part_md;
    m.n = h->npad;
    return m;
}

static LcArgs lc_args(ec_problem *h, int seq, double *part = nullptr)
{
    LcArgs l{};
    SeqDev *sd = h->seq_d + seq;
    l.A = basis_Q(h, seq);
    l.B = basis_KQ(h, seq);
    l.ld = h->ld;
    l.kp = &sd->ncol_md;
    l.cA = sd->cA;
    l.cB = sd->cB;
    l.a1 = &sd->a1;
    l.a2 = &sd->a2;
    l.part = part ? part : h->part_md;
    l.n = h->npad;
    return l;
}

static SmallArgs small_args(ec_problem *h, int seq, int op, const double *part,
                            ec_solve_info *info = nullptr)
{
    SmallArgs a{};
    a.seq = h->seq_d + seq;
    a.op = op;
    a.part = part;
    // values a dense step can read: SPE k <= cap, ncol_md <= cap + 1; POD
    // 2 npush <= 2 cap, count <= cap (loaded before the count is known)
    a.nvals = std::min(kMdStride, 2 * h->cap + 2);
    a.tol = h->dep_tol;
    a.info = info;
    return a;
}


// Arguments of the three launches of a start vector: x0 and r0 = b - K_n x0
// (into rb[0]) from the history of seq (eqs. 10, 14)
struct StartArgs {
    MdArgs m;
    SmallArgs s;
    LcArgs l;
};

static StartArgs seq_start_args(ec_problem *h, int seq, int method, const double *b,
                                const double *bscale, double *x0, ec_solve_info *info)
{
    SeqDev *sd = h->seq_d + seq;
    StartArgs a;
    a.m = md_args(h);
    a.m.A = basis_Q(h, seq);
    a.m.kp = method == EC_SV_POD ? &sd->count : &sd->k;
    a.m.B[0] = {b, bscale};
    a.m.nb = 1;
    a.s = small_args(h, seq, method == EC_SV_POD ? OP_POD_START : OP_SPE_START, h->part_md, info);
    a.l = lc_args(h, seq);
    a.l.v2 = {b, bscale};
    a.l.y1 = x0;
    a.l.y2 = h->rb[0];
    return a;
}

static void seq_start(ec_problem *h, int seq, int method, const double *b, const double *bscale,
                      double *x0, ec_solve_info *info)
{
    const StartArgs a = seq_start_args(h, seq, method, b, bscale, x0, info);
    multidot(a.m, h->st);
    small(a.s, h->st);
    lincomb(a.l, h->st);
}

// Arguments of the launches of a history push of solution x into seq, with
// scratch set `set` (0 or 1: two pushes may share launches).  SPE: two
// classical Gram-Schmidt passes against the orthogonal basis, the new column
// and its K_n product into their slots with (K_n + eta D^T D) t2 for the new
// column of Q^T (K_n + eta D^T D) Q (the grad-div term keeps the projection
// from amplifying the gradient part of the window), then the window downdate.
// POD: the snapshot and its K_n product into the ring slot, a Gram row.
struct PushArgs {
    MdArgs m, m2;
    LcArgs l1, l2;
    SlotArgs sa;
    RotArgs ro;
    SmallArgs s1, s2, s3, s4;   // s1-s3: the one-block form (batched SPE pushes, POD)
};

// fused: the SPE coefficient steps and the acceptance test run in the
// blocks of the kernels that apply them (one problem); otherwise as
// one-block steps (batched pushes: most of an instance's blocks have little
// work, and each would repeat the step's reduction)
static PushArgs seq_push_args(ec_problem *h, int seq, int method, const double *x, int set,
                              bool fused = true)
{
    double *w = set ? h->w_b : h->w, *t2 = set ? h->t2_b : h->t2;
    double *t3 = set ? h->t3_b : h->t3, *t4 = set ? h->t4_b : h->t4;
    double *part = set ? h->part_md_b : h->part_md;
    SeqDev *sd = h->seq_d + seq;
    double *Q = basis_Q(h, seq), *KQ = basis_KQ(h, seq);
    PushArgs a{};
    if (method == EC_SV_POD) {
        a.sa = SlotArgs{x, t3, KQ, Q, nullptr, &sd->slot_new, &sd->push_on, 0.0, nullptr, nullptr, 0.0};
        a.m = md_args(h, part);
        a.m.active = &sd->push_on;      // only a solution that is due
        a.m.A = Q;
        a.m.kp = &sd->npush;
        a.m.B[0] = {x, nullptr};
        a.m.B[1] = {t3, nullptr};
        a.m.nb = 2;
        a.s1 = small_args(h, seq, OP_POD_PUSH, part);
        return a;
    }
    a.m = md_args(h, part);
    a.m.A = Q;
    a.m.kp = &sd->k;
    a.m.a_extra = x;
    a.m.B[0] = {x, nullptr};
    a.m.nb = 1;
    a.m.active = &sd->push_on;     // only a solution that is due
    // the dense steps between the products run in the next kernel's blocks:
    // w = x - q c1 with c1 from q^T x (and the dots q^T w into the upper
    // half of the partials, which the product's values still occupy below),
    // x2 = w - q c2, then the acceptance test in the slot SpMV
    double *part_hi = part + (int64_t)kMaxWin * kMdBlocks;
    a.l1 = lc_args(h, seq, part_hi);
    a.l1.v1 = x;
    a.l1.y1 = w;
    a.l1.want_dots = 1;
    a.l1.pre_seq = sd;
    a.l1.pre_op = OP_SPE_PUSH1;
    a.l1.pin = part;
    a.l2 = a.l1;
    a.l2.v1 = w;
    a.l2.y1 = t2;
    a.l2.want_dots = 0;
    a.l2.pre_op = OP_SPE_PUSH2;
    a.l2.pin = part_hi;
    a.l2.part = part;
    a.sa = SlotArgs{t2, nullptr, KQ, Q, t4, &sd->slot_new, nullptr, h->seq_eta[seq],
                    sd, part, h->dep_tol};
    if (!fused) {
        a.s1 = small_args(h, seq, OP_SPE_PUSH1, part);
        a.s2 = small_args(h, seq, OP_SPE_PUSH2, part);
        a.s3 = small_args(h, seq, OP_SPE_PUSH3, part);
        for (LcArgs *l : {&a.l1, &a.l2}) {
            l->pre_seq = nullptr;
            l->active = &sd->active;
            l->part = part;
        }
        a.sa.pre_seq = nullptr;
        a.sa.active = &sd->active;
    }
    a.m2 = md_args(h, part);
    a.m2.A = Q;
    a.m2.kp = &sd->ncol_md;
    a.m2.B[0] = {t4, nullptr};
    a.m2.nb = 1;
    a.m2.active = &sd->accept;
    a.s4 = small_args(h, seq, OP_SPE_PUSH4, part);
    a.ro = RotArgs{Q, KQ, sd, h->ld, h->npad};
    return a;
}

// Append solution xs[i] to the history of sequence seqs[i] (n = 1 or 2
// independent sequences of one problem, same method) on stream st: every
// kernel of the push is one launch for both, each with its own scratch and
// partials (sets set0, set0 + 1).  Each push is gated on its sequence's
// push_on and clears it.
static void seq_push_n(ec_problem *h, int n, const int *seqs, int method,
                       const double *const *xs, hipStream_t st, int set0 = 0)
{
    PushArgs a[2];
    for (int i = 0; i < n; ++i) a[i] = seq_push_args(h, seqs[i], method, xs[i], set0 + i);
    const PushArgs *b = n == 2 ? &a[1] : nullptr;
    if (method == EC_SV_POD) {
        spmv_slots(h->g, h->ld, a[0].sa, st, b ? &b->sa : nullptr);
        multidot(a[0].m, st, b ? &b->m : nullptr);
        small(a[0].s1, st, b ? &b->s1 : nullptr);
        return;
    }
    multidot(a[0].m, st, b ? &b->m : nullptr);
    lincomb(a[0].l1, st, b ? &b->l1 : nullptr);
    lincomb(a[0].l2, st, b ? &b->l2 : nullptr);
    spmv_slots(h->g, h->ld, a[0].sa, st, b ? &b->sa : nullptr);
    multidot(a[0].m2, st, b ? &b->m2 : nullptr);
    small(a[0].s4, st, b ? &b->s4 : nullptr);
    rotate(a[0].ro, st, b ? &b->ro : nullptr);
}

// append solution x to the history of seq
static void seq_push(ec_problem *h, int seq, int method, const double *x)
{
    seq_push_n(h, 1, &seq, method, &x, h->st);
}

// Push the last coupling solution of launched graph steps if it is still due
// (they leave it for the next step's start); every call that reads or
// changes the histories, the solution buffers or what a push computes
// begins with this, so that pushes keep the order of eager steps.
static bool flush_pending(ec_problem *h)
{
    const int meth = h->pending_meth;
    h->pending_meth = -1;
    if (meth != EC_SV_SPE && meth != EC_SV_POD) return false;
    seq_push(h, EC_SEQ_CPL, meth, h->sc);
    return true;
}

// An executable captured step; for a problem's step with a start-vector
// history also the problem and the method (a launch leaves the step's
// coupling solution due for a push).
struct GraphBox {
    hipGraphExec_t ex;
    ec_problem *h;
    int meth;
};

// ------------------------------------------------------------- solve
static bool capturing(ec_problem *h)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(h->st, &cs);
    return cs != hipStreamCaptureStatusNone;
}

constexpr int kGraphMaxIters = 4096;

// Enqueue the iteration kernels of one CG solve.  Under graph capture a
// fixed budget of maxit iterations is recorded (each returns at once after
// convergence).  Eagerly, iterations go out in chunks and the host reads the
// device done flag of the previous chunk (pinned copy) while the next chunk
// runs; the first chunk is the previous iteration count of the sequence.
// want_cap > 0: where the tail is available, a captured solve issues at most
// that many iteration kernels, the last of them the tail (also without a
// sequence budget).
template <typename T>
static int32_t cg_iterate(ec_problem *h, const CgArgs<T> &a, int seq, bool hintable, int *n_issued,
                          bool *fin_done = nullptr, int want_cap = 0)
{
    if (fin_done) *fin_done = false;
    hipStream_t st = h->st;
    const int maxit = a.maxit;
    if (capturing(h)) {
        int budget = std::min(maxit, kGraphMaxIters);
        // the sequence budget caps the FP64 solve or each inner FP32 pass of
        // a refined solve; the tail finishes either
        int want = h->graph_iters[seq];
        const int tblocks = std::is_same<T, double>::value ? h->tail_blocks : h->tail_blocks_f;
        if (want_cap > 0 && tblocks > 0) want = want > 0 ? std::min(want, want_cap) : want_cap;
        const bool tail = want > 0 && want < maxit && tblocks > 0;
        if (want > 0) budget = std::min(budget, want);
        // with the tail, it runs the last budgeted iteration itself (the same
        // iteration body; one launch fewer when the solve is already done)
        const int kernels = tail ? budget - 1 : budget;
        for (int i = 0; i < kernels; ++i) cg_iter<T>(a, i, st);
        // rare long solves (cold start, a sudden change of the source) finish
        // in one persistent launch instead of failing at the budget
        if (tail) {
            // the tail also runs the solve's final step when the caller
            // takes it (one launch fewer)
            hipError_t e = cg_tail<T>(a, kernels, tblocks, st, fin_done != nullptr);
            if (e != hipSuccess)
                return fail(h, EC_ERR_HIP, "tail launch: %s", hipGetErrorString(e));
            if (fin_done) *fin_done = true;
        }
        *n_issued = budget;
        return launch_check(h, "cg (graph)");
    }
    int issued = 0, slot = 0, outstanding = -1;
    int chunk = std::max(1, (hintable ? h->hint[seq] : 16) + 1);
    bool first = true, done = false;
    while (!done && issued < maxit) {
        const int c = std::min(chunk, maxit - issued);
        for (int j = 0; j < c; ++j) cg_iter<T>(a, issued + j, st);
        issued += c;
        HIP_TRY(h, hipMemcpyAsync(h->pin + 8 * slot, &a.ctl[issued & 1].it, 4 * sizeof(int),
                                  hipMemcpyDeviceToHost, st));
        HIP_TRY(h, hipEventRecord(h->ev[slot], st));
        if (outstanding >= 0) {
            HIP_TRY(h, hipEventSynchronize(h->ev[outstanding]));
            done = h->pin[8 * outstanding + 1] != 0;
        }
        outstanding = slot;
        slot ^= 1;
        chunk = first ? std::max(2, chunk / 4) : std::min(2 * chunk, 256);
        first = false;
    }
    if (outstanding >= 0) {
        HIP_TRY(h, hipEventSynchronize(h->ev[outstanding]));
        if (hintable) h->hint[seq] = std::max(0, h->pin[8 * outstanding]);
    }
    *n_issued = issued;
    return launch_check(h, "cg");
}

template <typename T>
static void set_25(const ec_problem *h, CgArgs<T> &a)
{
    const bool on = h->t25 > 0 && h->cg_blocks == h->grid25;
    a.t25 = on ? h->t25 : 0;
    a.kb25 = h->kb25; a.nti25 = h->nti25; a.ntj25 = h->ntj25; a.ntk25 = h->ntk25;
}

static CgArgs<double> cg64_args(ec_problem *h, int seq, const double *b, const double *bscale,
                                double *x, const ec_solve_opts *o, ec_solve_info *info)
{
    CgArgs<double> a{};
    a.g = h->g;
    a.x = x;
    a.p = h->pv;
    for (int i = 0; i < 2; ++i) { a.rb[i] = h->rb[i]; a.wb[i] = h->wb[i]; a.sb[i] = h->sb[i]; }
    a.b = b;
    a.bscale = bscale;
    a.seq = h->seq_d + seq;
    a.rtol = o->rtol;
    a.maxit = o->maxit;
    a.ctl = h->cg_d;
    a.part = h->part_cg;
    a.info = info;
    a.ctrl = h->ctrl_d;
    a.seq_id = seq;
    a.accum = 0;
    a.skip = nullptr;
    a.tiles = h->tiles;
    a.blocks = h->cg_blocks;
    a.bar = h->bar;
    set_25(h, a);
    return a;
}

static void cg64_init(ec_problem *h, CgArgs<double> a, int mode)
{
    if (mode == START_X) {
        a.mode = START_X;
        cg_init<double>(a, h->st);
        a.mode = START_R2;
        cg_init<double>(a, h->st);
    } else {
        a.mode = mode;
        cg_init<double>(a, h->st);
    }
}

static int32_t run_cg64(ec_problem *h, int seq, int mode, const double *b, const double *bscale,
                        double *x, const ec_solve_opts *o, ec_solve_info *info)
{
    CgArgs<double> a = cg64_args(h, seq, b, bscale, x, o, info);
    // an SPE/POD start: its combination's residual sums (h->part_md) let the
    // init kernel stop a solve the start already solved
    if (mode == START_DEV) a.start_part = h->part_md;
    cg64_init(h, a, mode);
    int issued = 0;
    bool fin_done = false;
    int32_t rc = cg_iterate<double>(h, a, seq, true, &issued, &fin_done);
    if (rc) return rc;
    if (!fin_done) cg_fin<double>(a, issued, h->st);
    return launch_check(h, "cg fin");
}

// ------------------------------------------------ solve in outside scratch
// Bytes of device scratch that solve_scratch needs for this handle: the seven
// PCG vectors (r, w, s double buffered, p), two control records, the block
// partials and the tail kernel's barrier words.
int64_t ec::scratch_need(const ec_problem *h)
{
    const int64_t ld = align_up(h->npad, 64);
    return 7 * ld * 8 + align_up(2 * (int64_t)sizeof(CgCtl), kAlign) +
           align_up(2 * 4 * (int64_t)kMaxBlocks * 8, kAlign) +
           align_up((int64_t)kBarWords * kBarStride * sizeof(unsigned), kAlign);
}

// the limit stated in ec.h: the largest n_padded whose scratch fits the array
constexpr int64_t scratch_need_for(int64_t npad)
{
    return 7 * ((npad + 63) / 64 * 64) * 8 + (2 * (int64_t)sizeof(CgCtl) + 255) / 256 * 256 +
           (2 * 4 * (int64_t)kMaxBlocks * 8 + 255) / 256 * 256 +
           ((int64_t)kBarWords * kBarStride * (int64_t)sizeof(unsigned) + 255) / 256 * 256;
}
static_assert(scratch_need_for(EC_STATIC_MAX_NPAD) <= EC_STATIC_SCRATCH_BYTES &&
                  scratch_need_for(EC_STATIC_MAX_NPAD + 1) > EC_STATIC_SCRATCH_BYTES,
              "EC_STATIC_MAX_NPAD does not match the static scratch layout");

hipStream_t ec::bound_stream(const ec_problem *h) { return h && h->bound ? h->st : nullptr; }

// The FP64 PCG of ec_solve (ZERO or PREV start, sequence USER without
// history) with all of its scratch in the device buffer scr of `bytes`
// bytes instead of the handle's workspace; the handle's counters are left
// alone.  lookup: the status of the buffer's address lookup.
int32_t ec::solve_scratch(ec_problem *h, int32_t method, const double *b, double *x,
                          const ec_solve_opts *o, ec_solve_info *info, char *scr, int64_t bytes,
                          hipError_t lookup)
{
    NEED_BOUND(h);
    if (lookup != hipSuccess || !scr)
        return fail(h, EC_ERR_HIP, "address of the static scratch array: %s",
                    hipGetErrorString(lookup));
    flush_pending(h);
    if (!aligned(b) || !aligned(x) || !o)
        return fail(h, EC_ERR_ARG, "b, x must be 16-byte aligned device pointers; opts required");
    if (method != EC_SV_ZERO && method != EC_SV_PREV)
        return fail(h, EC_ERR_ARG, "the static-scratch solve starts from zero or from x");
    if (o->precision != EC_PREC_FP64)
        return fail(h, EC_ERR_ARG, "the static-scratch solve runs FP64 PCG");
    if (!(o->rtol > 0) || o->maxit < 0) return fail(h, EC_ERR_ARG, "need rtol > 0, maxit >= 0");
    const int64_t need = scratch_need(h);
    if (need > bytes)
        return fail(h, EC_ERR_ARG,
                    "grid too large for the static scratch: %lld bytes needed (n_padded %lld), "
                    "%lld available", (long long)need, (long long)h->npad, (long long)bytes);
    const int64_t ld = align_up(h->npad, 64);
    CgArgs<double> a = cg64_args(h, EC_SEQ_USER, b, nullptr, x, o, info);
    double *v = (double *)scr;
    for (int i = 0; i < 2; ++i) {
        a.rb[i] = v + (0 + i) * ld;
        a.wb[i] = v + (2 + i) * ld;
        a.sb[i] = v + (4 + i) * ld;
    }
    a.p = v + 6 * ld;
    char *q = scr + 7 * ld * 8;
    a.ctl = (CgCtl *)q;
    q += align_up(2 * (int64_t)sizeof(CgCtl), kAlign);
    a.part = (double *)q;
    q += align_up(2 * 4 * (int64_t)kMaxBlocks * 8, kAlign);
    a.bar = (unsigned *)q;
    a.seq = nullptr;
    a.ctrl = nullptr;
    cg64_init(h, a, method == EC_SV_ZERO ? START_ZERO : START_X);
    int issued = 0;
    bool fin_done = false;
    int32_t rc = cg_iterate<double>(h, a, EC_SEQ_USER, false, &issued, &fin_done);
    if (rc) return rc;
    if (!fin_done) cg_fin<double>(a, issued, h->st);
    return launch_check(h, "static-scratch solve");
}

// FP64 residual refinement around FP32 inner PCG solves of K_n d = r
static int32_t run_refined(ec_problem *h, int seq, const double *b, const double *bscale,
                           double *x, const ec_solve_opts *o, ec_solve_info *info)
{
    hipStream_t st = h->st;
    const int outer = o->outer_max > 0 ? o->outer_max : 8;
    refine_reset(h->ctrl_d, st);
    const double inner_rtol = o->inner_rtol > 0 ? o->inner_rtol : 1e-5;
    const bool eager = !capturing(h);
    for (int pass = 0; pass <= outer; ++pass) {
        refine_residual(h->g, b, bscale, x, h->frb[0], h->part_ref, h->ctrl_d, h->cg_blocks, st);
        refine_decide(h->part_ref, h->cg_blocks, h->ctrl_d, pass, outer, o->rtol, inner_rtol, info,
                      h->seq_d + seq, st);
        if (pass == outer) break;
        if (eager) {
            // stop issuing passes once the FP64 residual check has passed
            HIP_TRY(h, hipMemcpyAsync(h->pin + 16, &h->ctrl_d->refine_done, sizeof(int),
                                      hipMemcpyDeviceToHost, st));
            HIP_TRY(h, hipStreamSynchronize(st));
            if (h->pin[16]) break;
        }
        CgArgs<float> a{};
        a.g = h->g;
        a.x = h->fd;
        a.p = h->fpv;
        for (int i = 0; i < 2; ++i) { a.rb[i] = h->frb[i]; a.wb[i] = h->fwb[i]; a.sb[i] = h->fsb[i]; }
        a.b = h->frb[0];      // the FP32 residual is the right-hand side (read in init only)
        a.bscale = nullptr;
        a.mode = START_ZERO;
        a.seq = nullptr;
        a.rtol = inner_rtol;
        a.rtol_dev = &h->ctrl_d->refine_tol;    // set by refine_decide for this pass
        a.maxit = o->inner_maxit > 0 ? o->inner_maxit : 200;
        a.ctl = h->cg_d;
        a.part = h->part_cg;
        a.info = info;
        a.ctrl = h->ctrl_d;
        a.seq_id = seq;
        a.accum = 1;
        a.skip = &h->ctrl_d->refine_done;
        a.tiles = h->tiles;
        a.blocks = h->cg_blocks;
        a.bar = h->bar;
        set_25(h, a);
        cg_init<float>(a, st);
        int issued = 0;
        // captured: the first pass gets the sequence budget; a later pass is
        // a correction the first one rarely leaves (it is skipped once the
        // FP64 check has passed), so it issues one kernel and the tail
        int32_t rc = cg_iterate<float>(h, a, seq, false, &issued, nullptr, pass == 0 ? 0 : 2);
        if (rc) return rc;
        cg_fin<float>(a, issued, st);
        refine_update(x, h->fd, h->ctrl_d, h->npad, st);
    }
    refine_final(x, h->ctrl_d, h->npad, st);
    return launch_check(h, "refined solve");
}

// start vector of a solve (eqs. 10, 14 for SPE / POD) and the PCG start mode
static int32_t solve_prepare(ec_problem *h, int seq, int method, int window, int kmax,
                             double eps, const double *b, const double *bscale, double *x,
                             const ec_solve_opts *o, ec_solve_info *info, int *mode,
                             bool launch_start = true)
{
    if (o->precision != EC_PREC_FP64 && o->precision != EC_PREC_FP32_REFINED)
        return fail(h, EC_ERR_ARG, "unknown precision %d", o->precision);
    if (!(o->rtol > 0) || o->maxit < 0) return fail(h, EC_ERR_ARG, "need rtol > 0, maxit >= 0");
    if (method == EC_SV_ZERO) {
        *mode = START_ZERO;
    } else if (method == EC_SV_PREV) {
        *mode = START_X;
    } else if (method == EC_SV_SPE || method == EC_SV_POD) {
        if (window < 1 || window > h->cap)
            return fail(h, EC_ERR_ARG, "window must be 1..%d (the bound window_cap)", h->cap);
        seq_ensure(h, seq, method, window, kmax, eps);
        seq_eta_ensure(h, seq, method, spe_eta(h, o->precision));
        if (launch_start) seq_start(h, seq, method, b, bscale, x, info);
        *mode = START_DEV;
    } else {
        return fail(h, EC_ERR_ARG, "unknown start method %d", method);
    }
    return EC_OK;
}

static int32_t do_solve(ec_problem *h, int seq, int method, int window, int kmax, double eps,
                        const double *b, const double *bscale, double *x, const ec_solve_opts *o,
                        ec_solve_info *info, bool push)
{
    int mode = 0;
    int32_t rc;
    {
        Range r("start vector");
        rc = solve_prepare(h, seq, method, window, kmax, eps, b, bscale, x, o, info, &mode);
    }
    if (rc) return rc;
    {
        Range r("pcg");
        if (o->precision == EC_PREC_FP64) {
            rc = run_cg64(h, seq, mode, b, bscale, x, o, info);
        } else {
            if (mode == START_ZERO) fill(x, 0.0, h->npad, h->st);
            rc = run_refined(h, seq, b, bscale, x, o, info);
        }
    }
    if (rc != EC_OK) return rc;
    if (push && (method == EC_SV_SPE || method == EC_SV_POD)) {
        Range r("push");
        seq_push(h, seq, method, x);
    }
    return launch_check(h, "solve");
}

static bool valid_seq(int seq) { return seq >= 0 && seq < EC_NSEQ; }

extern "C" int32_t ec_solve(ec_handle h, int32_t seq, int32_t method, int32_t window,
                            const double *b, double *x, const ec_solve_opts *opts,
                            ec_solve_info *dev_info)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (!valid_seq(seq)) return fail(h, EC_ERR_ARG, "seq must be 0..%d", EC_NSEQ - 1);
    if (!aligned(b) || !aligned(x) || !opts)
        return fail(h, EC_ERR_ARG, "b, x must be 16-byte aligned device pointers; opts required");
    const int kmax = (h->seq_method[seq] == method && h->seq_win[seq] == window) ? h->seq_kmax[seq]
                                                                                  : window;
    const double eps = (h->seq_method[seq] == method && h->seq_win[seq] == window)
                           ? h->seq_eps[seq] : 1e-4;
    return do_solve(h, seq, method, window, kmax, eps, b, nullptr, x, opts, dev_info, true);
}

extern "C" int32_t ec_set_gauge_penalty(ec_handle h, double factor)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (!(factor >= 0.0) || !std::isfinite(factor))
        return fail(h, EC_ERR_ARG, "factor must be finite and >= 0");
    // histories built with another weight start anew at their next use
    h->gauge_rel = factor;
    return EC_OK;
}

extern "C" int32_t ec_set_pcg_kernel(ec_handle h, int32_t kind)
{
    NEED_BOUND(h);
    if (kind < -1 || kind > 1) return fail(h, EC_ERR_ARG, "kind must be -1, 0 or 1");
    h->t25 = 0;
    if (kind == 0 || (kind == -1 && !plan_25(h, false))) {
        h->cg_blocks = h->node_blocks;
        return EC_OK;
    }
    if (!plan_25(h, true)) {
        h->cg_blocks = h->node_blocks;
        return fail(h, EC_ERR_ARG, "the 2.5D kernel does not fit this grid");
    }
    h->cg_blocks = h->grid25;
    return EC_OK;
}

// One FP64 PCG iteration of the handle's current kernel, every iteration
// active (a zero-start solve of the source into scratch vectors).
static int32_t time_pcg_iteration(ec_problem *h, double *us)
{
    ec_solve_opts o{};
    o.rtol = 1e-300;
    o.maxit = 1 << 30;
    CgArgs<double> a = cg64_args(h, EC_SEQ_USER, h->xs_d, &h->ctrl_d->one, h->t4, &o, nullptr);
    a.ctrl = nullptr;
    cg64_init(h, a, START_ZERO);
    const int warm = 3, reps = 20;
    for (int it = 0; it < warm; ++it) cg_iter<double>(a, it, h->st);
    hipEvent_t e0, e1;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    HIP_TRY(h, hipEventRecord(e0, h->st));
    for (int it = warm; it < warm + reps; ++it) cg_iter<double>(a, it, h->st);
    HIP_TRY(h, hipEventRecord(e1, h->st));
    HIP_TRY(h, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us = 1e3 * ms / reps;
    return launch_check(h, "pcg timing");
}

extern "C" int32_t ec_tune_pcg(ec_handle h, const char *cache_path, int32_t *ti_out,
                               int32_t *kb_out, double *us_out)
{
    NEED_BOUND(h);
    flush_pending(h);
    std::string sig;
    {
        hipDeviceProp_t prop{};
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            sig += prop.gcnArchName;
        sig += ":" + std::to_string(h->g.nx) + "x" + std::to_string(h->g.ny) + "x" +
               std::to_string(h->g.nz);
    }
    auto apply = [&](int ti, int kb) -> bool {
        h->t25 = 0;
        if (ti == 0) {
            h->cg_blocks = h->node_blocks;
            return true;
        }
        if (!plan_25(h, true, ti, kb)) {
            h->cg_blocks = h->node_blocks;
            return false;
        }
        h->cg_blocks = h->grid25;
        return true;
    };
    int best_ti = -1, best_kb = 0;
    double best_us = 1e300;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char line[1024], key[900];
            int ti = 0, kb = 0;
            double us = 0.0;
            while (std::fgets(line, sizeof line, f))
                if (std::sscanf(line, "ec-pcg-tiling %899s %d %d %lf", key, &ti, &kb, &us) == 4 &&
                    sig == key) {
                    best_ti = ti; best_kb = kb; best_us = us;
                }
            std::fclose(f);
        }
        if (best_ti >= 0 && apply(best_ti, best_kb)) {
            if (ti_out) *ti_out = best_ti;
            if (kb_out) *kb_out = best_kb;
            if (us_out) *us_out = best_us;
            return EC_OK;
        }
    }
    best_ti = 0;
    best_us = 1e300;
    for (int ti : {0, 16, 32, 64})
        for (int kb : {4, 8, 16, 32}) {
            if (ti == 0 && kb != 4) continue;           // node-parallel: one candidate
            if (!apply(ti, kb)) continue;
            double us = 0.0;
            int32_t rc = time_pcg_iteration(h, &us);
            if (rc) return rc;
            if (us < best_us) {
                best_us = us; best_ti = ti; best_kb = ti ? h->kb25 : 0;
            }
        }
    apply(best_ti, best_kb);
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "ec-pcg-tiling %s %d %d %.4f\n", sig.c_str(), best_ti, best_kb, best_us);
            std::fclose(f);
        }
    }
    if (ti_out) *ti_out = best_ti;
    if (kb_out) *kb_out = best_kb;
    if (us_out) *us_out = best_us;
    return EC_OK;
}

extern "C" int32_t ec_set_dependency_tol(ec_handle h, double tol)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (!(tol > 0.0) || !(tol < 1.0)) return fail(h, EC_ERR_ARG, "tol must be in (0, 1)");
    h->dep_tol = tol;
    return EC_OK;
}

extern "C" int32_t ec_history_reset(ec_handle h, int32_t seq)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (!valid_seq(seq)) return fail(h, EC_ERR_ARG, "seq must be 0..%d", EC_NSEQ - 1);
    seq_reset(h->seq_d + seq, h->st);
    return launch_check(h, "history reset");
}

extern "C" int32_t ec_history_push(ec_handle h, int32_t seq, int32_t method, int32_t window,
                                   const double *x)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (!valid_seq(seq)) return fail(h, EC_ERR_ARG, "seq must be 0..%d", EC_NSEQ - 1);
    if (method != EC_SV_SPE && method != EC_SV_POD)
        return fail(h, EC_ERR_ARG, "history push needs SPE or POD");
    if (window < 1 || window > h->cap) return fail(h, EC_ERR_ARG, "window must be 1..%d", h->cap);
    if (!aligned(x)) return fail(h, EC_ERR_ARG, "x must be a 16-byte aligned device pointer");
    const int kmax = (h->seq_method[seq] == method && h->seq_win[seq] == window) ? h->seq_kmax[seq]
                                                                                  : window;
    const double eps = (h->seq_method[seq] == method && h->seq_win[seq] == window)
                           ? h->seq_eps[seq] : 1e-4;
    seq_ensure(h, seq, method, window, kmax, eps);
    seq_eta_ensure(h, seq, method, spe_eta(h, EC_PREC_FP64));
    seq_push_on(h->seq_d + seq, h->st);
    seq_push(h, seq, method, x);
    return launch_check(h, "history push");
}

extern "C" int32_t ec_start_vector(ec_handle h, int32_t seq, int32_t method, int32_t window,
                                   int32_t pod_kmax, double pod_eps, const double *b, double *x0,
                                   ec_solve_info *dev_info)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (!valid_seq(seq)) return fail(h, EC_ERR_ARG, "seq must be 0..%d", EC_NSEQ - 1);
    if (method != EC_SV_SPE && method != EC_SV_POD)
        return fail(h, EC_ERR_ARG, "start vector needs SPE or POD");
    if (window < 1 || window > h->cap) return fail(h, EC_ERR_ARG, "window must be 1..%d", h->cap);
    if (pod_kmax < 1 || pod_kmax > window || !(pod_eps >= 0))
        return fail(h, EC_ERR_ARG, "need 1 <= pod_kmax <= window and pod_eps >= 0");
    if (!aligned(b) || !aligned(x0))
        return fail(h, EC_ERR_ARG, "b, x0 must be 16-byte aligned device pointers");
    seq_ensure(h, seq, method, window, pod_kmax, pod_eps);
    seq_start(h, seq, method, b, nullptr, x0, dev_info);
    return launch_check(h, "start vector");
}

// ------------------------------------------------------------- apply
extern "C" int32_t ec_apply(ec_handle h, int32_t op, const double *x, double *y)
{
    NEED_BOUND(h);
    if (!aligned(x) || !aligned(y) || x == y)
        return fail(h, EC_ERR_ARG, "x, y must be distinct 16-byte aligned device pointers");
    hipStream_t st = h->st;
    int lo[3] = {0, 0, 0}, hi[3] = {h->g.nx, h->g.ny, h->g.nz};
    switch (op) {
    case EC_OP_KN:
        mask_copy(h->g, x, h->t4, 2, st);
        spmv(h->g, h->t4, y, lo, hi, st);
        break;
    case EC_OP_KCN_T:
        mask_copy(h->g, x, h->t4, 1, st);
        spmv(h->g, h->t4, y, lo, hi, st);
        break;
    case EC_OP_KC_KCN: {
        fill(y, 0.0, h->npad, st);
        UpdArgs u{};
        u.g = h->g; u.m = h->mats_d; u.cmat = h->cmat_d; u.cslot = h->cslot_d; u.minv = h->minv_d;
        u.nc = h->nc; u.A = x; u.xn = x; u.nustate = x; u.out = y; u.apply = 1;
        update_c(u, st);
        break;
    }
    default:
        return fail(h, EC_ERR_ARG, "unknown operator %d", op);
    }
    return launch_check(h, "apply");
}

// ------------------------------------------------ consistent M_c solves
static MassOp mass_op(const ec_problem *h) { return MassOp{h->m_idx_d, h->m_val_d, h->m_dinv_d, h->nc}; }

// basis-product and combination arguments over the mass sequence's compact
// columns (length n_c, stride ldc)
static MdArgs mass_md(ec_problem *h)
{
    MdArgs m{};
    m.ld = h->ldc;
    m.part = h->m_part_md;
    m.n = h->nc;
    m.A = h->m_hist;
    return m;
}

static LcArgs mass_lc(ec_problem *h, double *part)
{
    SeqDev *sd = h->mseq_d;
    LcArgs l{};
    l.A = h->m_hist;
    l.B = h->m_hist + (int64_t)(h->cap + 1) * h->ldc;
    l.ld = h->ldc;
    l.kp = &sd->ncol_md;
    l.cA = sd->cA;
    l.cB = sd->cB;
    l.a1 = &sd->a1;
    l.a2 = &sd->a2;
    l.part = part;
    l.n = h->nc;
    return l;
}

// Append y (compact, the last solution) to the mass sequence's SPE history:
// the push of seq_push_args (two Gram-Schmidt passes, coefficient steps in
// the combinations' blocks, the acceptance test in the slot product, window
// downdate) with M_c in place of K_n and no grad-div term.
static void mass_push(ec_problem *h, const double *y)
{
    hipStream_t st = h->st;
    SeqDev *sd = h->mseq_d;
    double *part = h->m_part_md, *part_hi = part + (int64_t)kMaxWin * kMdBlocks;
    double *Q = h->m_hist, *MQ = h->m_hist + (int64_t)(h->cap + 1) * h->ldc;
    MdArgs m = mass_md(h);
    m.kp = &sd->k;
    m.a_extra = y;
    m.B[0] = {y, nullptr};
    m.nb = 1;
    m.active = &sd->push_on;
    LcArgs l1 = mass_lc(h, part_hi);
    l1.v1 = y;
    l1.y1 = h->m_w;
    l1.want_dots = 1;
    l1.pre_seq = sd;
    l1.pre_op = OP_SPE_PUSH1;
    l1.pin = part;
    LcArgs l2 = l1;
    l2.v1 = h->m_w;
    l2.y1 = h->m_t2;
    l2.want_dots = 0;
    l2.pre_op = OP_SPE_PUSH2;
    l2.pin = part_hi;
    l2.part = part;
    MdArgs m2 = mass_md(h);
    m2.kp = &sd->ncol_md;
    m2.B[0] = {h->m_t4, nullptr};
    m2.nb = 1;
    m2.active = &sd->accept;
    SmallArgs s4{};
    s4.seq = sd;
    s4.op = OP_SPE_PUSH4;
    s4.part = part;
    s4.nvals = std::min(kMdStride, 2 * h->cap + 2);
    s4.tol = h->dep_tol;
    multidot(m, st);
    lincomb(l1, st);
    lincomb(l2, st);
    mass_slots(mass_op(h), h->ldc, h->m_t2, MQ, Q, h->m_t4, &sd->slot_new, sd, part, h->dep_tol,
               st);
    multidot(m2, st);
    small(s4, st);
    rotate(RotArgs{Q, MQ, sd, h->ldc, h->nc}, st);
}

// y = M_c^{-1} g (compact vectors) by Jacobi-PCG from zero or from the SPE
// start of the mass sequence (eq. 10 with M_c), then the push of y.  Eager
// solves poll the done flag in chunks; a captured solve issues mass_maxit
// iteration kernels (those after convergence return at once).
static int32_t mass_solve(ec_problem *h, const double *g, double *y, ec_solve_info *info)
{
    hipStream_t st = h->st;
    SeqDev *sd = h->mseq_d;
    const bool spe = h->mass_method == EC_SV_SPE;
    if (spe) {
        MdArgs m = mass_md(h);
        m.kp = &sd->k;
        m.B[0] = {g, nullptr};
        m.nb = 1;
        SmallArgs sa{};
        sa.seq = sd;
        sa.op = OP_SPE_START;
        sa.part = h->m_part_md;
        sa.nvals = std::min(kMdStride, 2 * h->cap + 2);
        sa.tol = h->dep_tol;
        sa.info = info;
        LcArgs l = mass_lc(h, h->m_part_md);
        l.v2 = {g, nullptr};
        l.y1 = y;
        l.y2 = h->m_rb[0];
        multidot(m, st);
        small(sa, st);
        lincomb(l, st);
    }
    MassCg a{};
    a.M = mass_op(h);
    a.x = y;
    a.b = g;
    a.p = h->m_p;
    for (int i = 0; i < 2; ++i) { a.rb[i] = h->m_rb[i]; a.wb[i] = h->m_wb[i]; a.sb[i] = h->m_sb[i]; }
    a.ctl = h->m_ctl;
    a.part = h->m_part;
    a.blocks = mass_blocks(h->nc);
    a.rtol = h->mass_rtol;
    a.maxit = h->mass_maxit;
    a.mode = spe ? START_DEV : START_ZERO;
    a.seq = spe ? sd : nullptr;
    a.info = info;
    a.ctrl = h->ctrl_d;
    mass_cg_init(a, st);
    int issued = 0;
    if (capturing(h)) {
        for (; issued < a.maxit; ++issued) mass_cg_iter(a, issued, st);
    } else {
        int chunk = std::max(1, h->mass_hint + 1), outstanding = -1, slot = 0;
        bool done = false;
        while (!done && issued < a.maxit) {
            const int c = std::min(chunk, a.maxit - issued);
            for (int j = 0; j < c; ++j) mass_cg_iter(a, issued + j, st);
            issued += c;
            HIP_TRY(h, hipMemcpyAsync(h->pin + 8 * slot, &a.ctl[issued & 1].it, 4 * sizeof(int),
                                      hipMemcpyDeviceToHost, st));
            HIP_TRY(h, hipEventRecord(h->ev[slot], st));
            if (outstanding >= 0) {
                HIP_TRY(h, hipEventSynchronize(h->ev[outstanding]));
                done = h->pin[8 * outstanding + 1] != 0;
            }
            outstanding = slot;
            slot ^= 1;
            chunk = std::min(2 * chunk, 64);
        }
        if (outstanding >= 0) {
            HIP_TRY(h, hipEventSynchronize(h->ev[outstanding]));
            h->mass_hint = std::max(0, h->pin[8 * outstanding]);
        }
    }
    mass_cg_fin(a, issued, st);
    if (spe) mass_push(h, y);
    return launch_check(h, "mass solve");
}

extern "C" int32_t ec_set_mass(ec_handle h, int32_t kind, int32_t method, int32_t window,
                               double rtol, int32_t maxit)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (kind != EC_MASS_LUMPED && kind != EC_MASS_CONSISTENT)
        return fail(h, EC_ERR_ARG, "unknown conductivity matrix kind %d", kind);
    if (method != EC_SV_ZERO && method != EC_SV_SPE)
        return fail(h, EC_ERR_ARG, "M_c solves start from zero or from SPE");
    if (method == EC_SV_SPE && (window < 1 || window > h->cap))
        return fail(h, EC_ERR_ARG, "window must be 1..%d", h->cap);
    if (!(rtol > 0) || maxit < 1) return fail(h, EC_ERR_ARG, "need rtol > 0, maxit >= 1");
    h->mass_kind = kind;
    h->mass_method = method;
    h->mass_win = method == EC_SV_SPE ? window : 1;
    h->mass_rtol = rtol;
    h->mass_maxit = maxit;
    seq_config(h->mseq_d, EC_SV_SPE, h->mass_win, h->mass_win, 1e-4, h->m_hscale, h->st);
    seq_reset(h->mseq_d, h->st);
    return launch_check(h, "set mass");
}

extern "C" int32_t ec_mass_apply(ec_handle h, const double *x, double *y)
{
    NEED_BOUND(h);
    if (!aligned(x) || !aligned(y) || x == y)
        return fail(h, EC_ERR_ARG, "x, y: distinct 16-byte aligned device pointers");
    gather_c(h->cslot_d, h->nc, x, h->m_g, h->st);
    mass_apply(mass_op(h), h->m_g, h->m_y, h->st);
    scatter_c(h->cslot_d, h->nc, h->m_y, y, h->st);
    return launch_check(h, "mass apply");
}

extern "C" int32_t ec_mass_solve(ec_handle h, const double *g, double *y, ec_solve_info *dev_info)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (!aligned(g) || !aligned(y))
        return fail(h, EC_ERR_ARG, "g, y must be 16-byte aligned device pointers");
    if (!h->nc) return fail(h, EC_ERR_ARG, "no conducting edges");
    Range range("mass solve");
    gather_c(h->cslot_d, h->nc, g, h->m_g, h->st);
    int32_t rc = mass_solve(h, h->m_g, h->m_y, dev_info);
    if (rc) return rc;
    scatter_c(h->cslot_d, h->nc, h->m_y, y, h->st);
    return launch_check(h, "mass solve");
}

extern "C" int32_t ec_mass_counters(ec_handle h, int64_t *solves, int64_t *iters)
{
    NEED_BOUND(h);
    Ctrl c{};
    HIP_TRY(h, hipMemcpyAsync(&c, h->ctrl_d, sizeof c, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(h, hipStreamSynchronize(h->st));
    if (solves) *solves = c.mass_solves;
    if (iters) *iters = c.mass_iters;
    return EC_OK;
}

// -------------------------------------------------------------- step
// One explicit Euler step: source solve, coupled right-hand side, coupling
// solve, history pushes, state update.  split (a captured step with a
// start-vector history): the pushes run on the side stream beside the other
// sequence's work, each on the second scratch set.  First the push of the
// previous step's coupling solution (skipped when it was already made, see
// SeqDev::push_on) beside this step's source start and solve, then this
// step's source push beside the coupling start and solve; this step's
// coupling solution stays due for the next step or a flush.  The pushes read
// only their sequence's state and solution, so the results are those of the
// eager order.
static int32_t step_impl(ec_problem *h, int64_t m, double dt, double *A, const ec_step_opts *o,
                         ec_solve_info *info, bool split = false)
{
    Range step_range("step");
    hipStream_t st = h->st, sd = h->side;
    const int meth = o->start_method;
    split = split && (meth == EC_SV_SPE || meth == EC_SV_POD);
    if (split) {
        Range r("push");
        const int seq = EC_SEQ_CPL;
        const double *x = h->sc;
        HIP_TRY(h, hipEventRecord(h->sev[0], st));
        HIP_TRY(h, hipStreamWaitEvent(sd, h->sev[0], 0));
        seq_push_n(h, 1, &seq, meth, &x, sd, 1);
        HIP_TRY(h, hipEventRecord(h->sev[1], sd));
    }
    step_begin(h->ctrl_d, m, h->wf, h->amp, h->freq, h->tau, h->ramp, dt, st, h->adapt_lam,
               h->adapt_safety);
    int32_t rc;
    {
        Range r("source solve");
        rc = do_solve(h, EC_SEQ_SRC, meth, o->window, o->pod_kmax, o->pod_eps, h->xs_d,
                      &h->ctrl_d->scale, h->sj, &o->solve, info, false);
    }
    if (rc) return rc;
    if (split) {
        Range r("push");
        const int seq = EC_SEQ_SRC;
        const double *x = h->sj;
        HIP_TRY(h, hipEventRecord(h->sev[2], st));
        HIP_TRY(h, hipStreamWaitEvent(sd, h->sev[2], 0));
        seq_push_n(h, 1, &seq, meth, &x, sd, 1);
        HIP_TRY(h, hipEventRecord(h->sev[3], sd));
    }
    {
        Range r("update");
        UpdArgs u{};
        u.g = h->g; u.m = h->mats_d; u.cmat = h->cmat_d; u.cslot = h->cslot_d; u.minv = h->minv_d;
        u.nc = h->nc; u.A = A; u.sj = h->sj; u.sc = h->sc; u.out = h->ac; u.dt = dt; u.apply = 0;
        u.ctrl = h->ctrl_d;
        if (h->mass_kind == EC_MASS_CONSISTENT && h->nc) {
            // eq. 6 with a consistent M_c: g on C, M_c y = g (its own sequence),
            // a_c^m = a_c^{m-1} - dt y
            u.gout = h->m_g;
            update_c(u, st);
            rc = mass_solve(h, h->m_g, h->m_y, nullptr);
            if (rc) return rc;
            mass_axpy(h->cslot_d, h->nc, A, h->m_y, h->ctrl_d, h->ac, st);
        } else {
            update_c(u, st);
        }
        if (h->has_cond) spmv(h->g, h->ac, h->bcpl, h->band_lo, h->band_hi, st);
    }
    if (split) HIP_TRY(h, hipStreamWaitEvent(st, h->sev[1], 0));
    {
        Range r("coupling solve");
        rc = do_solve(h, EC_SEQ_CPL, meth, o->window, o->pod_kmax, o->pod_eps, h->bcpl, nullptr,
                      h->sc, &o->solve, info ? info + 1 : nullptr, false);
    }
    if (rc) return rc;
    if (split) {
        HIP_TRY(h, hipStreamWaitEvent(st, h->sev[3], 0));
    } else if (meth == EC_SV_SPE || meth == EC_SV_POD) {
        Range r("push");
        // both histories grow in the same launches: the source history is
        // next read by the source solve of the following step
        const int seqs[2] = {EC_SEQ_SRC, EC_SEQ_CPL};
        const double *xs[2] = {h->sj, h->sc};
        seq_push_n(h, 2, seqs, meth, xs, st);
    }
    {
        Range r("finish state");
        finish_state(h->g, A, h->ac, h->sj, h->sc, h->ctrl_d, 1, st);
    }
    return launch_check(h, "step");
}

static int32_t check_step_args(ec_problem *h, double dt, const double *A, const ec_step_opts *o)
{
    if (!aligned(A) || !o) return fail(h, EC_ERR_ARG, "A must be aligned; opts required");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(h, EC_ERR_ARG, "dt must be positive");
    if (!h->adapt_lam && h->cfl_lam > 0.0 && dt * h->cfl_lam > 2.0)
        return fail(h, EC_ERR_CFL,
                    "dt %.6g above the explicit Euler bound 2/lambda_max = %.6g of the last "
                    "ec_cfl (eq. 8)", dt, 2.0 / h->cfl_lam);
    const int m = o->start_method;
    if (m < EC_SV_ZERO || m > EC_SV_POD) return fail(h, EC_ERR_ARG, "unknown start method");
    if ((m == EC_SV_SPE || m == EC_SV_POD) &&
        (o->window < 1 || o->window > h->cap || o->pod_kmax < 1 || o->pod_kmax > o->window ||
         !(o->pod_eps >= 0)))
        return fail(h, EC_ERR_ARG, "window 1..%d, 1 <= pod_kmax <= window, pod_eps >= 0", h->cap);
    return EC_OK;
}

extern "C" int32_t ec_step(ec_handle h, int64_t m, double dt, double *A, const ec_step_opts *opts,
                           ec_solve_info *dev_info)
{
    NEED_BOUND(h);
    flush_pending(h);
    int32_t rc = check_step_args(h, dt, A, opts);
    if (rc) return rc;
    return step_impl(h, m, dt, A, opts, dev_info);
}

extern "C" int32_t ec_run(ec_handle h, int64_t m0, int64_t nsteps, double dt, double *A,
                          const ec_step_opts *opts, ec_solve_info *dev_info)
{
    NEED_BOUND(h);
    flush_pending(h);
    int32_t rc = check_step_args(h, dt, A, opts);
    if (rc) return rc;
    if (nsteps < 0) return fail(h, EC_ERR_ARG, "nsteps must be >= 0");
    for (int64_t s = 0; s < nsteps; ++s) {
        rc = step_impl(h, m0 + 1 + s, dt, A, opts, dev_info ? dev_info + 2 * s : nullptr);
        if (rc) return rc;
    }
    return EC_OK;
}

static int32_t set_state_impl(ec_problem *h, const double *A, const ec_solve_opts *opts);

extern "C" int32_t ec_set_state(ec_handle h, const double *A, const ec_solve_opts *opts)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (!aligned(A) || !opts) return fail(h, EC_ERR_ARG, "A must be aligned; opts required");
    Range range("set state");
    return set_state_impl(h, A, opts);
}

static int32_t set_state_impl(ec_problem *h, const double *A, const ec_solve_opts *opts)
{
    hipStream_t st = h->st;
    fill(h->ac, 0.0, h->npad, st);
    copy_c(h->cslot_d, h->nc, A, h->ac, st);
    fill(h->bcpl, 0.0, h->npad, st);
    if (h->has_cond) spmv(h->g, h->ac, h->bcpl, h->band_lo, h->band_hi, st);
    int32_t rc = do_solve(h, EC_SEQ_CPL, EC_SV_ZERO, 1, 1, 0.0, h->bcpl, nullptr, h->sc, opts,
                          nullptr, false);
    if (rc) return rc;
    fill(h->sj, 0.0, h->npad, st);
    fill(&h->ctrl_d->t, 0.0, 1, st);     // the clock of adaptive steps starts at 0
    for (int s = 0; s < EC_NSEQ; ++s) seq_reset(h->seq_d + s, st);
    seq_reset(h->mseq_d, st);
    HIP_TRY(h, hipStreamSynchronize(st));
    return launch_check(h, "set state");
}

extern "C" int32_t ec_set_step(ec_handle h, int64_t m)
{
    NEED_BOUND(h);
    if (m < 0) return fail(h, EC_ERR_ARG, "m must be >= 0");
    Ctrl c{};
    HIP_TRY(h, hipMemcpyAsync(&c, h->ctrl_d, sizeof c, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(h, hipStreamSynchronize(h->st));
    c.step = m;
    HIP_TRY(h, hipMemcpyAsync(h->ctrl_d, &c, sizeof c, hipMemcpyHostToDevice, h->st));
    HIP_TRY(h, hipStreamSynchronize(h->st));
    return EC_OK;
}

// ---------------------------------------------------------- counters
extern "C" int32_t ec_counters(ec_handle h, int64_t *n_steps, int64_t *iters_src,
                               int64_t *iters_cpl, int64_t *iters_adj, int32_t *worst_status)
{
    NEED_BOUND(h);
    Ctrl c{};
    HIP_TRY(h, hipMemcpyAsync(&c, h->ctrl_d, sizeof c, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(h, hipStreamSynchronize(h->st));
    if (n_steps) *n_steps = c.n_steps;
    if (iters_src) *iters_src = c.iters[EC_SEQ_SRC];
    if (iters_cpl) *iters_cpl = c.iters[EC_SEQ_CPL];
    if (iters_adj) *iters_adj = c.iters[EC_SEQ_ADJ];
    if (worst_status) *worst_status = c.worst;
    return EC_OK;
}

extern "C" int32_t ec_counters_reset(ec_handle h)
{
    NEED_BOUND(h);
    Ctrl c{};
    HIP_TRY(h, hipMemcpyAsync(&c, h->ctrl_d, sizeof c, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(h, hipStreamSynchronize(h->st));
    c.n_steps = 0;
    for (int s = 0; s < EC_NSEQ; ++s) c.iters[s] = 0;
    c.mass_solves = 0;
    c.mass_iters = 0;
    c.worst = EC_OK;
    HIP_TRY(h, hipMemcpyAsync(h->ctrl_d, &c, sizeof c, hipMemcpyHostToDevice, h->st));
    HIP_TRY(h, hipStreamSynchronize(h->st));
    return EC_OK;
}

// -------------------------------------------------------------- CFL
// Power method on M_c^{-1} K_S (eq. 8) in the M_c inner product:
//   s = K_n^+ K_cn^T v ;  g = [K_nu(A) (v (+) -s)]_C = K_S v ;
//   lambda = v^T g (v M_c-normalised) ; v <- M_c^{-1} g.
extern "C" int32_t ec_cfl(ec_handle h, const double *A, int32_t power_iters, double rtol,
                          double *lambda_max)
{
    NEED_BOUND(h);
    if (!aligned(A) || !lambda_max || power_iters < 1 || !(rtol > 0))
        return fail(h, EC_ERR_ARG, "bad arguments");
    if (h->nc == 0) return fail(h, EC_ERR_ARG, "no conducting edges");
    Range range("cfl power method");
    hipStream_t st = h->st;
    std::vector<double> v(h->nc), gv(h->nc);
    uint32_t s = 12345u;
    for (int t = 0; t < h->nc; ++t) {
        s = s * 1664525u + 1013904223u;
        v[t] = (double)(s >> 8) / 16777216.0 - 0.5;
    }
    ec_solve_opts o{rtol, 1000000, EC_PREC_FP64, 0.0, 0, 0};
    double lam = 0.0;
    for (int it = 0; it < power_iters; ++it) {
        double nrm = 0.0;
        for (int t = 0; t < h->nc; ++t) nrm += v[t] * v[t] / h->minv[t];
        nrm = std::sqrt(nrm);
        for (int t = 0; t < h->nc; ++t) v[t] /= nrm;
        HIP_TRY(h, hipMemcpyAsync(h->cvec_d, v.data(), (size_t)h->nc * 8, hipMemcpyHostToDevice, st));
        fill(h->t4, 0.0, h->npad, st);
        scatter_c(h->cslot_d, h->nc, h->cvec_d, h->t4, st);
        fill(h->w, 0.0, h->npad, st);
        spmv(h->g, h->t4, h->w, h->band_lo, h->band_hi, st);
        int32_t rc = run_cg64(h, EC_SEQ_USER, START_ZERO, h->w, nullptr, h->t2, &o, nullptr);
        if (rc) return rc;
        // g = [K_nu(A) (v (+) -s)]_C with v on C (t4) and -s on N (t3)
        negate(h->t2, h->t3, h->npad, st);
        UpdArgs u{};
        u.g = h->g; u.m = h->mats_d; u.cmat = h->cmat_d; u.cslot = h->cslot_d; u.minv = h->minv_d;
        u.nc = h->nc; u.A = h->t4; u.sj = nullptr; u.sc = nullptr; u.xn = h->t3;
        u.nustate = A; u.apply = 1;
        // g into t2's conducting slots (apply mode writes C entries only)
        u.out = h->t2;
        update_c(u, st);
        gather_c(h->cslot_d, h->nc, h->t2, h->cvec_d, st);
        HIP_TRY(h, hipMemcpyAsync(gv.data(), h->cvec_d, (size_t)h->nc * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(h, hipStreamSynchronize(st));
        double num = 0.0;
        for (int t = 0; t < h->nc; ++t) num += v[t] * gv[t];
        lam = num;
        for (int t = 0; t < h->nc; ++t) v[t] = gv[t] * h->minv[t];
    }
    *lambda_max = lam;
    if (std::isfinite(lam) && lam > 0.0) h->cfl_lam = lam;
    return launch_check(h, "cfl");
}

// ------------------------------------------------ implicit Euler / Newton
// P^-1 J v for column v (compact) into out: v on C and 0 on N (i_v), cell
// records of J_N(a) in direction v, s = K_n^+ K_cn^T v (zero start, the
// USER sequence), u = v (+) -s (i_u), (J_N - S) v by the edge pass, then
// v + dt M_c^-1 (J_N - S) v.
static int32_t newton_matvec(ec_problem *h, const double *v, double dt, const ec_solve_opts *so,
                             double *out)
{
    hipStream_t st = h->st;
    const int nc = h->nc;
    scatter_c(h->cslot_d, nc, v, h->i_v, st);
    jn_cell(h->g, h->mats_d, h->cmat_d, h->i_a, h->i_v, h->cellv_d, h->bblo, h->bbhi, st);
    spmv(h->g, h->i_v, h->i_b, h->band_lo, h->band_hi, st);
    int32_t rc = do_solve(h, EC_SEQ_USER, EC_SV_ZERO, 1, 1, 0.0, h->i_b, nullptr, h->i_s, so,
                          nullptr, false);
    if (rc) return rc;
    negate(h->i_s, h->i_u, h->npad, st);
    scatter_c(h->cslot_d, nc, v, h->i_u, st);
    jn_edge(h->g, h->cslot_d, nc, h->cellv_d, h->i_u, h->i_a, h->i_jv, st);
    gm_precond(nc, v, h->i_jv, h->minv_d, dt, out, st);
    return EC_OK;
}

static int32_t read_dev(ec_problem *h, const void *src, size_t bytes, int slot)
{
    HIP_TRY(h, hipMemcpyAsync(h->pin + 24 + slot, src, bytes, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(h, hipStreamSynchronize(h->st));
    return EC_OK;
}

// One implicit Euler step m (the paper's reference method): Newton on the
// Schur form of eq. (3) (a_n eliminated as in eqs. 4-5b):
//   F(a) = M_c (a - a_old)/dt + g(a, s_j - s_c(a)),  s_j = K_n^+ j^m,
//   s_c(a) = K_n^+ K_cn^T a, g the conducting rows of K(nu(a)) (eq. 6's g),
// J d = -F with J = M_c/dt + J_N(a) - S by GMRES(m) left-preconditioned with
// (M_c/dt)^-1, a += d, until ||F|| <= newton_rtol ||F(a_old)||.  The source
// and coupling solves run on the SRC and CPL sequences with the options'
// start vector (consecutive Newton iterates converge, so SPE extrapolates
// their s_c); the products' K_n^+ solves start from zero.  Host control
// reads ||F|| after each Newton iteration and GMRES's convergence flag after
// each Arnoldi step; all arithmetic runs in kernels.
extern "C" int32_t ec_implicit_step(ec_handle h, int64_t m, double dt, double *A,
                                    const ec_implicit_opts *o, ec_implicit_info *info)
{
    NEED_BOUND(h);
    Range range("implicit step");
    flush_pending(h);
    if (!aligned(A) || !o || !(dt > 0) || !std::isfinite(dt))
        return fail(h, EC_ERR_ARG, "need an aligned A, opts and dt > 0");
    if (!(o->newton_rtol > 0) || o->max_newton < 1 || o->gmres_m < 1 || o->gmres_m > kGmMax ||
        o->gmres_max < 1 || !(o->gmres_rtol > 0) || !(o->inner_rtol > 0))
        return fail(h, EC_ERR_ARG, "newton_rtol, gmres_rtol, inner_rtol > 0; max_newton, "
                                   "gmres_max >= 1; 1 <= gmres_m <= %d", kGmMax);
    const int meth = o->start_method;
    if (meth < EC_SV_ZERO || meth > EC_SV_POD ||
        ((meth == EC_SV_SPE || meth == EC_SV_POD) && (o->window < 1 || o->window > h->cap)))
        return fail(h, EC_ERR_ARG, "start method and window 1..%d", h->cap);
    if (!h->has_cond) return fail(h, EC_ERR_ARG, "the implicit step needs a conductor");
    if (h->mass_kind != EC_MASS_LUMPED || h->adapt_lam)
        return fail(h, EC_ERR_STATE, "the implicit step uses the lumped M_c and a fixed dt");
    if (capturing(h)) return fail(h, EC_ERR_STATE, "the implicit step is not captured");
    hipStream_t st = h->st;
    const int nc = h->nc;
    const ec_solve_opts so{o->inner_rtol, 1000000, EC_PREC_FP64, 0.0, 0, 0};
    const int win = (meth == EC_SV_SPE || meth == EC_SV_POD) ? o->window : 1;
    step_begin(h->ctrl_d, m, h->wf, h->amp, h->freq, h->tau, h->ramp, dt, st);
    int32_t rc = do_solve(h, EC_SEQ_SRC, meth, win, win, 1e-4, h->xs_d, &h->ctrl_d->scale, h->sj,
                          &so, nullptr, false);
    if (rc) return rc;
    if (meth == EC_SV_SPE || meth == EC_SV_POD) seq_push(h, EC_SEQ_SRC, meth, h->sj);
    adj_cell_init(h->cellv_d, h->ncell, h->mats.nu0, st);   // air cells: nu0, no d nu
    fill(h->i_a, 0.0, h->npad, st);
    copy_c(h->cslot_d, nc, A, h->i_a, st);
    gather_c(h->cslot_d, nc, A, h->i_aold, st);
    fill(h->i_v, 0.0, h->npad, st);
    fill(h->i_b, 0.0, h->npad, st);
    int newton = 0, gm_total = 0, kn = 1;
    double f0 = -1.0, fn = 0.0;
    const int64_t ldc = h->ldc;
    GmDev *gm = h->gm_d;
    for (;;) {
        // s_c(a) and F(a)
        spmv(h->g, h->i_a, h->bcpl, h->band_lo, h->band_hi, st);
        rc = do_solve(h, EC_SEQ_CPL, meth, win, win, 1e-4, h->bcpl, nullptr, h->sc, &so, nullptr,
                      false);
        if (rc) return rc;
        if (meth == EC_SV_SPE || meth == EC_SV_POD) seq_push(h, EC_SEQ_CPL, meth, h->sc);
        ++kn;
        UpdArgs u{};
        u.g = h->g; u.m = h->mats_d; u.cmat = h->cmat_d; u.cslot = h->cslot_d; u.minv = h->minv_d;
        u.nc = nc; u.A = h->i_a; u.sj = h->sj; u.sc = h->sc; u.gout = h->i_F; u.ctrl = h->ctrl_d;
        update_c(u, st);
        newton_residual(nc, h->cslot_d, h->i_a, h->i_aold, h->minv_d, dt, h->i_F, st);
        nrm2_fin(h->i_pn, nrm2_part(nc, h->i_F, h->i_pn, st), h->i_norm, st);
        double nv = 0.0;
        rc = read_dev(h, h->i_norm, 8, 0);
        if (rc) return rc;
        std::memcpy(&nv, h->pin + 24, 8);
        fn = nv;
        if (f0 < 0.0) f0 = fn;
        if (!(fn > o->newton_rtol * f0) || newton >= o->max_newton) break;
        // GMRES(m): P^-1 J d = -P^-1 F from d = 0
        fill(h->i_x, 0.0, nc, st);
        gm_precond(nc, nullptr, h->i_F, h->minv_d, dt, h->i_t, st);     // -P^-1 F
        HIP_TRY(h, hipMemcpyAsync(h->i_w, h->i_t, (size_t)nc * 8, hipMemcpyDeviceToDevice, st));
        bool first = true;
        for (;;) {
            gm_begin(gm, h->i_pn, nrm2_part(nc, h->i_w, h->i_pn, st), first ? 1 : 0, o->gmres_rtol,
                     st);
            first = false;
            LcArgs l0{};
            l0.A = h->i_V; l0.ld = ldc; l0.kp = &gm->ncol; l0.cA = gm->coef; l0.a1 = &gm->a1;
            l0.v1 = h->i_w; l0.slot = &gm->slot; l0.part = h->i_part; l0.n = nc;
            lincomb(l0, st);
            rc = read_dev(h, &gm->conv, 4, 4);
            if (rc) return rc;
            if (h->pin[28]) break;
            int jn = 0;
            bool conv = false;
            for (int j = 0; j < o->gmres_m && gm_total < o->gmres_max; ++j) {
                rc = newton_matvec(h, h->i_V + (int64_t)j * ldc, dt, &so, h->i_w);
                if (rc) return rc;
                ++kn;
                MdArgs md{};
                md.A = h->i_V; md.ld = ldc; md.kfix = j + 1; md.B[0] = {h->i_w, nullptr}; md.nb = 1;
                md.part = h->i_part; md.n = nc;
                multidot(md, st);
                gm_orth1(gm, h->i_part, j, st);
                LcArgs l1{};
                l1.A = h->i_V; l1.ld = ldc; l1.kp = &gm->ncol; l1.cA = gm->coef; l1.a1 = &gm->a1;
                l1.v1 = h->i_w; l1.y1 = h->i_w; l1.want_dots = 1; l1.part = h->i_part; l1.n = nc;
                lincomb(l1, st);
                gm_orth2(gm, h->i_part, j, st);
                LcArgs l2 = l1;
                l2.y1 = nullptr;
                l2.slot = &gm->slot;
                l2.want_dots = 0;
                lincomb(l2, st);
                ++jn;
                ++gm_total;
                rc = read_dev(h, &gm->conv, 4, 4);
                if (rc) return rc;
                if (h->pin[28]) {
                    conv = true;
                    break;
                }
            }
            gm_solve(gm, jn, st);
            LcArgs lx{};
            lx.A = h->i_V; lx.ld = ldc; lx.kp = &gm->ncol; lx.cA = gm->coef; lx.a1 = &gm->a1;
            lx.v1 = h->i_x; lx.y1 = h->i_x; lx.part = h->i_part; lx.n = nc;
            lincomb(lx, st);
            if (conv || gm_total >= o->gmres_max) break;
            // restart on the true residual -P^-1 F - P^-1 J d
            rc = newton_matvec(h, h->i_x, dt, &so, h->i_w);
            if (rc) return rc;
            ++kn;
            vsub(nc, h->i_t, h->i_w, h->i_w, st);
        }
        newton_update(nc, h->cslot_d, h->i_x, h->i_a, st);
        ++newton;
    }
    // the new state: a on C, s_j - s_c(a) on N (s_c of the last Newton iterate)
    finish_state(h->g, A, h->i_a, h->sj, h->sc, h->ctrl_d, 1, st);
    rc = launch_check(h, "implicit step");
    if (rc) return rc;
    if (info) {
        info->newton_iters = newton;
        info->gmres_iters = gm_total;
        info->kn_solves = kn;
        info->status = std::isfinite(fn) ? (fn > o->newton_rtol * f0 ? EC_ERR_NOT_CONVERGED : EC_OK)
                                         : EC_ERR_NONFINITE;
        info->res0 = f0;
        info->res = fn;
    }
    HIP_TRY(h, hipStreamSynchronize(st));
    return EC_OK;
}

// ------------------------------------------------- stability estimate
// Power method for the explicit Euler bound (eq. 8 and the power method named
// after it) with the reluctivity at state A: B = (X^T - S) M_c^{-1},
// X = J_N(A) (jacobian) or K_c(nu(A)); B is the transpose of
// M_c^{-1} (X - S), so it has its eigenvalues.  Per iteration, with the unit
// iterate v (compact): w = M_c^{-1} v on C; cell records of X at A (and w
// for J_N); s = K_n^+ K_cn^T w, one solve of the EC_SEQ_USER sequence started
// as `method` says (the right-hand sides of consecutive iterations converge:
// SPE extrapolates them); y = [C^T (M_nu C u + q)]_C with u = w on C and -s
// on N, i.e. X^T w - S w; lambda = ||y||, v <- y / lambda on the device.
// Scratch: the second push set (w_b, t2_b..t4_b), free outside captures.
extern "C" int32_t ec_cfl_estimate(ec_handle h, const double *A, int32_t iters, double rtol,
                                   int32_t method, int32_t window, int32_t jacobian,
                                   double *lambda_dev, double *rec_dev)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (!aligned(A) || !lambda_dev || iters < 1 || !(rtol > 0))
        return fail(h, EC_ERR_ARG, "need aligned A, lambda_dev, iters >= 1, rtol > 0");
    if (method != EC_SV_ZERO && method != EC_SV_PREV && method != EC_SV_SPE)
        return fail(h, EC_ERR_ARG, "inner solves start from zero, the previous or an SPE vector");
    if (method == EC_SV_SPE && (window < 1 || window > h->cap))
        return fail(h, EC_ERR_ARG, "window must be 1..%d", h->cap);
    if (h->nc == 0) return fail(h, EC_ERR_ARG, "no conducting edges");
    if (capturing(h)) return fail(h, EC_ERR_STATE, "the estimate is not captured");
    hipStream_t st = h->st;
    const int nc = h->nc;
    double *wpad = h->t2_b, *upad = h->t3_b, *bpad = h->t4_b, *spad = h->w_b;
    adj_cell_init(h->cellv_d, h->ncell, h->mats.nu0, st);
    fill(wpad, 0.0, h->npad, st);
    fill(bpad, 0.0, h->npad, st);
    fill(spad, 0.0, h->npad, st);
    power_init(nc, h->cvec2_d, st);
    const int seq = EC_SEQ_USER;
    const int win = method == EC_SV_SPE ? window : 1;
    if (method == EC_SV_SPE) {
        seq_ensure(h, seq, method, win, win, 1e-4);
        seq_eta_ensure(h, seq, method, spe_eta(h, EC_PREC_FP64));
    }
    seq_reset(h->seq_d + seq, st);
    const ec_solve_opts o{rtol, 1000000, EC_PREC_FP64, 0.0, 0, 0};
    for (int it = 0; it < iters; ++it) {
        adj_w(h->cslot_d, nc, h->cvec2_d, h->minv_d, wpad, st);
        if (jacobian || it == 0)
            adj_cell(h->g, h->mats_d, h->cmat_d, A, jacobian ? wpad : nullptr, h->cellv_d, 1,
                     h->bblo, h->bbhi, h->part_cell, st);
        if (h->has_cond) spmv(h->g, wpad, bpad, h->band_lo, h->band_hi, st);
        int32_t rc = do_solve(h, seq, method, win, win, 1e-4, bpad, nullptr, spad, &o, nullptr,
                              true);
        if (rc) return rc;
        negate(spad, upad, h->npad, st);
        adj_w(h->cslot_d, nc, h->cvec2_d, h->minv_d, upad, st);
        adj_edge(h->g, h->cslot_d, nc, h->cellv_d, upad, h->cvec_d, st);
        power_norm(nc, h->cvec_d, h->cvec2_d, lambda_dev, rec_dev ? rec_dev + 2 * it : nullptr,
                   st);
    }
    return launch_check(h, "stability estimate");
}

extern "C" int32_t ec_set_adaptive_dt(ec_handle h, const double *lambda_dev, double safety)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (lambda_dev && (!(safety > 0.0) || !(safety <= 1.0) ||
                       ((uintptr_t)lambda_dev % 8) != 0))
        return fail(h, EC_ERR_ARG, "need 0 < safety <= 1 and an 8-byte aligned device scalar");
    h->adapt_lam = lambda_dev;
    h->adapt_safety = lambda_dev ? safety : 0.5;
    return EC_OK;
}

extern "C" int32_t ec_clock(ec_handle h, int64_t *m, double *t, double *dt)
{
    NEED_BOUND(h);
    Ctrl c{};
    HIP_TRY(h, hipMemcpyAsync(&c, h->ctrl_d, sizeof c, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(h, hipStreamSynchronize(h->st));
    if (m) *m = c.step;
    if (t) *t = c.t;
    if (dt) *dt = c.dt;
    return EC_OK;
}

// ------------------------------------------------------------ graphs

// ------------------------------------------------------------ materials
// M_sigma of every conducting edge from the current material table (the
// conducting edge set itself is fixed at create: sigma stays positive).
static void conductivities(ec_problem *h, const int *mat_filter, std::vector<double> *out)
{
    const int nx = h->g.nx, ny = h->g.ny;
    const double hh[3] = {h->g.hx, h->g.hy, h->g.hz};
    out->assign(h->nc, 0.0);
    for (int t = 0; t < h->nc; ++t) {
        const int64_t e = h->cslot[t];
        const int c = (int)(e / h->S);
        const int64_t nd = e - (int64_t)c * h->S;
        const int i = (int)(nd % (nx + 1)), j = (int)((nd / (nx + 1)) % (ny + 1));
        const int k = (int)(nd / ((int64_t)(nx + 1) * (ny + 1)));
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        const double quarter = hh[a1] * hh[a2] / 4.0 / hh[c];
        double sum = 0.0;
        for (int d1 = -1; d1 <= 0; ++d1)
            for (int d2 = -1; d2 <= 0; ++d2) {
                int cc[3] = {i, j, k};
                cc[a1] += d1;
                cc[a2] += d2;
                const int m = h->cmat[((int64_t)cc[2] * ny + cc[1]) * nx + cc[0]];
                if (mat_filter) sum += (m == *mat_filter) ? 1.0 : 0.0;
                else sum += h->mats.sig[m];
            }
        (*out)[t] = sum * quarter;
    }
}

extern "C" int32_t ec_set_material(ec_handle h, int32_t mat_id, const ec_material *m)
{
    NEED_BOUND(h);
    flush_pending(h);
    if (mat_id < 1 || mat_id >= h->mats.n || !m)
        return fail(h, EC_ERR_ARG, "mat_id must be 1..%d", h->mats.n - 1);
    if (!(m->sigma > 0) || !std::isfinite(m->sigma) || !(m->k1 >= 0) || !std::isfinite(m->k1) ||
        !std::isfinite(m->k2) || !(m->k3 > 0) || !std::isfinite(m->k3))
        return fail(h, EC_ERR_ARG, "need sigma > 0, k1 >= 0, k3 > 0 and finite k2");
    h->cfl_lam = 0.0;   // the bound of eq. 8 moves with sigma and nu
    h->mats.sig[mat_id] = m->sigma;
    h->mats.k1[mat_id] = m->k1;
    h->mats.k2[mat_id] = m->k2;
    h->mats.k3[mat_id] = m->k3;
    mass_build(h);
    {
        int32_t rc = mass_upload(h);
        if (rc) return rc;
        seq_config(h->mseq_d, EC_SV_SPE, h->mass_win, h->mass_win, 1e-4, h->m_hscale, h->st);
        seq_reset(h->mseq_d, h->st);
    }
    std::vector<double> ms;
    conductivities(h, nullptr, &ms);
    for (int t = 0; t < h->nc; ++t) h->minv[t] = 1.0 / ms[t];
    hipStream_t st = h->st;
    HIP_TRY(h, hipMemcpyAsync(h->mats_d, &h->mats, sizeof(Mats), hipMemcpyHostToDevice, st));
    if (h->nc)
        HIP_TRY(h, hipMemcpyAsync(h->minv_d, h->minv.data(), (size_t)h->nc * 8,
                                  hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipStreamSynchronize(st));
    return EC_OK;
}

// -------------------------------------------------------------- adjoint
// Workspace of a forward/backward pair: one checkpoint per segment of
// `every` steps (a_c, s_c, s_j, and the source and coupling histories with
// their small-matrix state, so that a recomputed segment is bitwise the
// forward one), the states of one segment, and the adjoint's own vectors.
struct AdjWs {
    int64_t n_ckpt = 0, ck_bytes = 0, hist_bytes = 0;
    char *ck = nullptr;
    double *seg = nullptr;                                   // (every+1) x nc
    double *mu_a = nullptr, *mu_b = nullptr, *dnext = nullptr, *jt = nullptr, *phi = nullptr;
    double *wpad = nullptr, *apad = nullptr, *upad = nullptr, *badj = nullptr, *sadj = nullptr;
    double *aseg = nullptr, *cellv = nullptr, *part = nullptr, *acc = nullptr;
};

static int64_t adj_layout(const ec_problem *h, int64_t M, int every, char *base, AdjWs *w)
{
    int64_t off = 0;
    auto take = [&](int64_t bytes) -> char * {
        const int64_t o = off;
        off = align_up(off + bytes, kAlign);
        return base ? base + o : nullptr;
    };
    const int64_t ld = align_up(h->npad, 64), nc = std::max(h->nc, 1);
    w->n_ckpt = (M + every - 1) / every;
    w->hist_bytes = 2 * (int64_t)(h->cap + 1) * ld * 8;
    w->ck_bytes = align_up(nc * 8, kAlign) + 2 * ld * 8 + 2 * align_up(sizeof(SeqDev), kAlign) +
                  2 * w->hist_bytes;
    w->ck = take(w->n_ckpt * w->ck_bytes);
    w->seg = (double *)take((int64_t)(every + 1) * nc * 8);
    double **cvec[] = {&w->mu_a, &w->mu_b, &w->dnext, &w->jt, &w->phi};
    for (double **v : cvec) *v = (double *)take(nc * 8);
    double **pvec[] = {&w->wpad, &w->apad, &w->upad, &w->badj, &w->sadj, &w->aseg};
    for (double **v : pvec) *v = (double *)take(ld * 8);
    w->cellv = (double *)take(h->ncell * 5 * 8);
    w->part = (double *)take((std::max<int64_t>(h->ncell, nc) / 256 + 2) * 8);
    w->acc = (double *)take(4 * 8);
    return off;
}

struct CkPtrs {
    double *ac, *sc, *sj;
    SeqDev *seq[2];
    double *hist[2];
};

static CkPtrs ckpt(const ec_problem *h, const AdjWs &w, int64_t k)
{
    const int64_t ld = align_up(h->npad, 64), nc = std::max(h->nc, 1);
    char *p = w.ck + k * w.ck_bytes;
    CkPtrs c{};
    c.ac = (double *)p;
    p += align_up(nc * 8, kAlign);
    c.sc = (double *)p;
    p += ld * 8;
    c.sj = (double *)p;
    p += ld * 8;
    for (int q = 0; q < 2; ++q) {
        c.seq[q] = (SeqDev *)p;
        p += align_up(sizeof(SeqDev), kAlign);
    }
    for (int q = 0; q < 2; ++q) {
        c.hist[q] = (double *)p;
        p += w.hist_bytes;
    }
    return c;
}

static int32_t ckpt_copy(ec_problem *h, const AdjWs &w, int64_t k, const double *ac, bool save)
{
    const CkPtrs c = ckpt(h, w, k);
    hipStream_t st = h->st;
    const size_t vb = (size_t)h->npad * 8;
    const int seqs[2] = {EC_SEQ_SRC, EC_SEQ_CPL};
    if (save) {
        if (h->nc)
            HIP_TRY(h, hipMemcpyAsync(c.ac, ac, (size_t)h->nc * 8, hipMemcpyDeviceToDevice, st));
        HIP_TRY(h, hipMemcpyAsync(c.sc, h->sc, vb, hipMemcpyDeviceToDevice, st));
        HIP_TRY(h, hipMemcpyAsync(c.sj, h->sj, vb, hipMemcpyDeviceToDevice, st));
        for (int q = 0; q < 2; ++q) {
            HIP_TRY(h, hipMemcpyAsync(c.seq[q], h->seq_d + seqs[q], sizeof(SeqDev),
                                      hipMemcpyDeviceToDevice, st));
            HIP_TRY(h, hipMemcpyAsync(c.hist[q], h->hist[seqs[q]], w.hist_bytes,
                                      hipMemcpyDeviceToDevice, st));
        }
    } else {
        HIP_TRY(h, hipMemcpyAsync(h->sc, c.sc, vb, hipMemcpyDeviceToDevice, st));
        HIP_TRY(h, hipMemcpyAsync(h->sj, c.sj, vb, hipMemcpyDeviceToDevice, st));
        for (int q = 0; q < 2; ++q) {
            HIP_TRY(h, hipMemcpyAsync(h->seq_d + seqs[q], c.seq[q], sizeof(SeqDev),
                                      hipMemcpyDeviceToDevice, st));
            HIP_TRY(h, hipMemcpyAsync(h->hist[seqs[q]], c.hist[q], w.hist_bytes,
                                      hipMemcpyDeviceToDevice, st));
        }
    }
    return EC_OK;
}

extern "C" int32_t ec_adjoint_sizes(ec_handle h, int64_t n_steps, int32_t checkpoint_every,
                                    int64_t *bytes)
{
    NEED_BOUND(h);
    if (n_steps < 1 || checkpoint_every < 1 || !bytes)
        return fail(h, EC_ERR_ARG, "need n_steps >= 1, checkpoint_every >= 1, bytes");
    AdjWs w;
    *bytes = adj_layout(h, n_steps, checkpoint_every, nullptr, &w);
    return EC_OK;
}

static int32_t adj_args(ec_problem *h, int64_t n_steps, double dt, int32_t every,
                        const ec_step_opts *opts, void *ws, int64_t bytes, double *A, AdjWs *w)
{
    int32_t rc = check_step_args(h, dt, A ? A : h->ac, opts);
    if (rc) return rc;
    if (!h->has_cond) return fail(h, EC_ERR_ARG, "the adjoint needs a conductor");
    if (h->adapt_lam)
        return fail(h, EC_ERR_STATE, "the adjoint runs fixed steps: ec_set_adaptive_dt(h, NULL, 0)");
    if (h->mass_kind != EC_MASS_LUMPED)
        return fail(h, EC_ERR_STATE, "the adjoint uses the lumped (diagonal) M_c");
    if (n_steps < 1 || every < 1) return fail(h, EC_ERR_ARG, "need n_steps >= 1, every >= 1");
    if (!ws || ((uintptr_t)ws % kAlign) != 0)
        return fail(h, EC_ERR_ARG, "adjoint workspace must be 256-byte aligned");
    const int64_t need = adj_layout(h, n_steps, every, (char *)ws, w);
    if (bytes < need) return fail(h, EC_ERR_ARG, "adjoint workspace too small (%lld < %lld)",
                                  (long long)bytes, (long long)need);
    return EC_OK;
}

extern "C" int32_t ec_adjoint_forward(ec_handle h, int64_t n_steps, double dt,
                                      int32_t checkpoint_every, const ec_step_opts *opts,
                                      void *adj_ws, int64_t adj_bytes, double *A, double *loss)
{
    NEED_BOUND(h);
    Range range("adjoint forward");
    flush_pending(h);
    AdjWs w;
    int32_t rc = adj_args(h, n_steps, dt, checkpoint_every, opts, adj_ws, adj_bytes, A, &w);
    if (rc) return rc;
    hipStream_t st = h->st;
    const int nc = h->nc;
    rc = set_state_impl(h, A, &opts->solve);           // a^0 from A; s_c, empty histories
    if (rc) return rc;
    adj_zero(w.acc, 4, st);
    double *prev = w.seg, *cur = w.seg + std::max(nc, 1);
    gather_c(h->cslot_d, nc, A, prev, st);
    for (int64_t m = 1; m <= n_steps; ++m) {
        if ((m - 1) % checkpoint_every == 0) {
            rc = ckpt_copy(h, w, (m - 1) / checkpoint_every, prev, true);
            if (rc) return rc;
        }
        rc = step_impl(h, m, dt, A, opts, nullptr);
        if (rc) return rc;
        gather_c(h->cslot_d, nc, A, cur, st);
        const int nb = adj_loss(nc, cur, prev, h->minv_d, dt, w.part, st);
        adj_accum(w.part, nb, 1.0, w.acc, st);
        std::swap(prev, cur);
    }
    if (loss) HIP_TRY(h, hipMemcpyAsync(loss, w.acc, 8, hipMemcpyDeviceToDevice, st));
    double chk = 0.0;
    HIP_TRY(h, hipMemcpyAsync(&chk, w.acc, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(h, hipStreamSynchronize(st));
    if (!std::isfinite(chk))
        return fail(h, EC_ERR_NONFINITE, "adjoint forward: the run diverged (loss %g); dt above "
                                         "the stability bound of eq. (8)?", chk);
    h->adj_ws = adj_ws;
    h->adj_steps = n_steps;
    h->adj_every = checkpoint_every;
    h->adj_dt = dt;
    return launch_check(h, "adjoint forward");
}

extern "C" int32_t ec_adjoint_backward(ec_handle h, int64_t n_steps, double dt,
                                       int32_t checkpoint_every, const ec_step_opts *opts,
                                       void *adj_ws, int64_t adj_bytes, int32_t mat_id,
                                       double *grads)
{
    NEED_BOUND(h);
    Range range("adjoint backward");
    flush_pending(h);
    AdjWs w;
    int32_t rc = adj_args(h, n_steps, dt, checkpoint_every, opts, adj_ws, adj_bytes, nullptr, &w);
    if (rc) return rc;
    if (h->adj_ws != adj_ws || h->adj_steps != n_steps || h->adj_every != checkpoint_every ||
        h->adj_dt != dt)
        return fail(h, EC_ERR_STATE, "ec_adjoint_forward with the same workspace, n_steps, "
                                     "checkpoint_every and dt first");
    if (mat_id < 1 || mat_id >= h->mats.n)
        return fail(h, EC_ERR_ARG, "mat_id must be 1..%d", h->mats.n - 1);
    if (!grads) return fail(h, EC_ERR_ARG, "grads is NULL");
    hipStream_t st = h->st;
    const int nc = h->nc, every = checkpoint_every;
    const int64_t M = n_steps;
    // dM_c/dsigma of the material: quarter dual faces of its cells per edge
    std::vector<double> phi;
    conductivities(h, &mat_id, &phi);
    HIP_TRY(h, hipMemcpyAsync(w.phi, phi.data(), (size_t)nc * 8, hipMemcpyHostToDevice, st));
    adj_zero(w.acc, 4, st);
    adj_cell_init(w.cellv, h->ncell, h->mats.nu0, st);
    fill(w.wpad, 0.0, h->npad, st);
    fill(w.apad, 0.0, h->npad, st);
    fill(w.badj, 0.0, h->npad, st);
    fill(w.aseg, 0.0, h->npad, st);
    fill(w.mu_b, 0.0, nc, st);
    fill(w.dnext, 0.0, nc, st);
    const int meth = opts->start_method;
    if (meth == EC_SV_SPE || meth == EC_SV_POD) {
        seq_ensure(h, EC_SEQ_ADJ, meth, opts->window, opts->pod_kmax, opts->pod_eps);
        seq_eta_ensure(h, EC_SEQ_ADJ, meth, spe_eta(h, opts->solve.precision));
    }
    seq_reset(h->seq_d + EC_SEQ_ADJ, st);
    double *mu_next = w.mu_b, *mu_cur = w.mu_a;
    for (int64_t k = w.n_ckpt - 1; k >= 0; --k) {
        const int64_t m0 = k * every, m1 = std::min<int64_t>(M, m0 + every);
        // recompute the segment from its checkpoint
        rc = ckpt_copy(h, w, k, nullptr, false);
        if (rc) return rc;
        const CkPtrs c = ckpt(h, w, k);
        if (nc) HIP_TRY(h, hipMemcpyAsync(w.seg, c.ac, (size_t)nc * 8, hipMemcpyDeviceToDevice, st));
        scatter_c(h->cslot_d, nc, w.seg, w.aseg, st);
        for (int64_t m = m0 + 1; m <= m1; ++m) {
            rc = step_impl(h, m, dt, w.aseg, opts, nullptr);
            if (rc) return rc;
            gather_c(h->cslot_d, nc, w.aseg, w.seg + (m - m0) * (int64_t)nc, st);
        }
        // adjoint steps m1 .. m0+1
        for (int64_t m = m1; m > m0; --m) {
            const double *am = w.seg + (m - m0) * (int64_t)nc;
            const double *am1 = w.seg + (m - m0 - 1) * (int64_t)nc;
            int nb;
            if (m == M) {
                nb = adj_mu(nc, am, am1, nullptr, w.dnext, h->minv_d, w.phi, nullptr, dt, 1,
                            mu_cur, w.part, st);
            } else {
                // w = M_c^{-1} mu_{m+1}; cell pass at a^m (and the k1 term of step m+1)
                adj_w(h->cslot_d, nc, mu_next, h->minv_d, w.wpad, st);
                scatter_c(h->cslot_d, nc, am, w.apad, st);
                const int nbc = adj_cell(h->g, h->mats_d, h->cmat_d, w.apad, w.wpad, w.cellv,
                                         mat_id, h->bblo, h->bbhi, w.part, st);
                adj_accum(w.part, nbc, -dt, w.acc + 2, st);
                // S w = K_cn K_n^+ K_cn^T w through one solve of the adjoint sequence
                spmv(h->g, w.wpad, w.badj, h->band_lo, h->band_hi, st);
                rc = do_solve(h, EC_SEQ_ADJ, meth, opts->window, opts->pod_kmax, opts->pod_eps,
                              w.badj, nullptr, w.sadj, &opts->solve, nullptr, true);
                if (rc) return rc;
                negate(w.sadj, w.upad, h->npad, st);
                adj_w(h->cslot_d, nc, mu_next, h->minv_d, w.upad, st);
                adj_edge(h->g, h->cslot_d, nc, w.cellv, w.upad, w.jt, st);
                nb = adj_mu(nc, am, am1, mu_next, w.dnext, h->minv_d, w.phi, w.jt, dt, 0, mu_cur,
                            w.part, st);
            }
            adj_accum(w.part, nb, 1.0, w.acc + 1, st);
            std::swap(mu_cur, mu_next);
        }
    }
    // k1 term of step 1: w_1 = M_c^{-1} mu_1 at a^0 (the first segment's start)
    adj_w(h->cslot_d, nc, mu_next, h->minv_d, w.wpad, st);
    scatter_c(h->cslot_d, nc, w.seg, w.apad, st);
    const int nbc = adj_cell(h->g, h->mats_d, h->cmat_d, w.apad, w.wpad, w.cellv, mat_id, h->bblo,
                             h->bbhi, w.part, st);
    adj_accum(w.part, nbc, -dt, w.acc + 2, st);
    HIP_TRY(h, hipMemcpyAsync(grads, w.acc + 1, 16, hipMemcpyDeviceToDevice, st));
    double chk[2] = {0.0, 0.0};
    HIP_TRY(h, hipMemcpyAsync(chk, w.acc + 1, 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(h, hipStreamSynchronize(st));
    if (!std::isfinite(chk[0]) || !std::isfinite(chk[1]))
        return fail(h, EC_ERR_NONFINITE, "adjoint backward: non-finite gradient");
    return launch_check(h, "adjoint backward");
}


// ---------------------------------------------------------------- batch
// Independent problems of uneven size (their own grid, materials and dt)
// advanced together on one stream.  Start vectors, the nonlinear update and
// the histories run as each problem's own kernels; the PCG iterations of all
// solves run in one launch per iteration (k_cg_iter_batch), each instance on
// its own slice of the grid with exactly the single-instance arithmetic.
// Start vectors and history pushes of all instances run as one launch per
// kernel from device tables of per-instance arguments (one block row each).
struct BasisTab {
    MdArgs *m_start, *m, *m2;
    SmallArgs *s_start, *s1, *s2, *s3, *s4;
    LcArgs *l_start, *l1, *l2;
    SlotTab *sa;
    RotArgs *ro;
};

struct ec_batch_s {
    std::vector<ec_problem *> inst;
    hipStream_t st = nullptr;
    CgArgs<double> *tab_d[2] = {};                 // per sequence: SRC, CPL
    std::vector<CgArgs<double>> tab[2];
    BasisTab btab[2];                              // per sequence, device tables
    int slot_tpx = 1;                              // slot SpMV grid of the largest instance
    // per-instance step control, conducting update, coupling right-hand
    // side and state assembly (device tables) and their largest grids
    StepArgs *step_tab = nullptr;
    UpdArgs *upd_tab = nullptr;
    BoxTab *box_tab = nullptr;
    FinArgs *fin_tab = nullptr;
    int nc_max = 0, box_tpx = 0;
    int64_t npad_max = 0;
    int *inst_d = nullptr, *off_d = nullptr, *flag_d = nullptr;
    int total_blocks = 0, max_blocks = 0;
    int tiles_per_block = 1;
    bool one_tile = true;                          // every instance: one tile per block
    int tail_blocks = 0;                           // grid of the batched tail (0: none)
};

static int64_t batch_layout(const std::vector<ec_problem *> &hs, char *base, ec_batch_s *b)
{
    int64_t off = 0;
    auto take = [&](int64_t bytes) -> char * {
        const int64_t o = off;
        off = align_up(off + bytes, kAlign);
        return base ? base + o : nullptr;
    };
    const int64_t n = (int64_t)hs.size();
    int64_t maxb = 0;
    for (ec_problem *h : hs) maxb += std::min<int64_t>(align_up(h->tiles, 8), kMaxBlocks);
    CgArgs<double> *t0 = (CgArgs<double> *)take(n * sizeof(CgArgs<double>));
    CgArgs<double> *t1 = (CgArgs<double> *)take(n * sizeof(CgArgs<double>));
    int *im = (int *)take(maxb * 4);
    int *of = (int *)take(n * 4);
    int *fl = (int *)take(64);
    BasisTab bt[2];
    for (BasisTab &t : bt) {
        t.m_start = (MdArgs *)take(n * sizeof(MdArgs));
        t.m = (MdArgs *)take(n * sizeof(MdArgs));
        t.m2 = (MdArgs *)take(n * sizeof(MdArgs));
        t.s_start = (SmallArgs *)take(n * sizeof(SmallArgs));
        t.s2 = (SmallArgs *)take(n * sizeof(SmallArgs));
        t.s3 = (SmallArgs *)take(n * sizeof(SmallArgs));
        t.s1 = (SmallArgs *)take(n * sizeof(SmallArgs));
        t.s4 = (SmallArgs *)take(n * sizeof(SmallArgs));
        t.l_start = (LcArgs *)take(n * sizeof(LcArgs));
        t.l1 = (LcArgs *)take(n * sizeof(LcArgs));
        t.l2 = (LcArgs *)take(n * sizeof(LcArgs));
        t.sa = (SlotTab *)take(n * sizeof(SlotTab));
        t.ro = (RotArgs *)take(n * sizeof(RotArgs));
    }
    StepArgs *stp = (StepArgs *)take(n * sizeof(StepArgs));
    UpdArgs *upd = (UpdArgs *)take(n * sizeof(UpdArgs));
    BoxTab *box = (BoxTab *)take(n * sizeof(BoxTab));
    FinArgs *fin = (FinArgs *)take(n * sizeof(FinArgs));
    if (b) {
        b->step_tab = stp;
        b->upd_tab = upd;
        b->box_tab = box;
        b->fin_tab = fin;
        b->btab[0] = bt[0];
        b->btab[1] = bt[1];
        b->tab_d[0] = t0;
        b->tab_d[1] = t1;
        b->inst_d = im;
        b->off_d = of;
        b->flag_d = fl;
        b->max_blocks = (int)maxb;
    }
    return off;
}

// PCG grid of each instance for a tiles-per-block factor, and the block map
static int32_t batch_apply_tiles(ec_batch_s *b, int f)
{
    std::vector<int> im, of;
    for (size_t i = 0; i < b->inst.size(); ++i) {
        ec_problem *h = b->inst[i];
        const int64_t nb = std::max<int64_t>(8, std::min<int64_t>(align_up((h->tiles + f - 1) / f, 8),
                                                                  kMaxBlocks));
        h->cg_blocks = (int)nb;
        of.push_back((int)im.size());
        for (int64_t q = 0; q < nb; ++q) im.push_back((int)i);
    }
    b->total_blocks = (int)im.size();
    b->tiles_per_block = f;
    b->one_tile = true;
    for (ec_problem *h : b->inst)
        if ((h->cg_blocks >> 3) < ((h->tiles + 7) >> 3) || h->g.px > kHaloMax) b->one_tile = false;
    ec_problem *h0 = b->inst[0];
    HIP_TRY(h0, hipMemcpyAsync(b->inst_d, im.data(), im.size() * 4, hipMemcpyHostToDevice, b->st));
    HIP_TRY(h0, hipMemcpyAsync(b->off_d, of.data(), of.size() * 4, hipMemcpyHostToDevice, b->st));
    HIP_TRY(h0, hipStreamSynchronize(b->st));
    return EC_OK;
}

// per-instance PCG, start-vector and history-push arguments of the source /
// coupling solves (device tables); the sequences are configured first, so
// the tables carry the current grad-div weights
static int32_t batch_tables(ec_batch_s *b, const ec_step_opts *so, const double *dt,
                            double *const *A)
{
    const ec_solve_opts *o = &so->solve;
    const int meth = so->start_method;
    const bool basis = meth == EC_SV_SPE || meth == EC_SV_POD;
    ec_problem *h0 = b->inst[0];
    const size_t ni = b->inst.size();
    {
        std::vector<StepArgs> stp(ni);
        std::vector<UpdArgs> upd(ni);
        std::vector<BoxTab> box(ni);
        std::vector<FinArgs> fin(ni);
        b->nc_max = 0;
        b->box_tpx = 0;
        b->npad_max = 0;
        for (size_t i = 0; i < ni; ++i) {
            ec_problem *h = b->inst[i];
            stp[i] = StepArgs{h->ctrl_d, h->wf,  h->amp,        h->freq,         h->tau,
                              h->ramp,   dt[i], h->adapt_lam, h->adapt_safety};
            UpdArgs &u = upd[i];
            u = UpdArgs{};
            u.g = h->g; u.m = h->mats_d; u.cmat = h->cmat_d; u.cslot = h->cslot_d;
            u.minv = h->minv_d; u.nc = h->nc; u.A = A[i]; u.sj = h->sj; u.sc = h->sc;
            u.out = h->ac; u.dt = dt[i]; u.apply = 0; u.ctrl = h->ctrl_d;
            BoxTab &bx = box[i];
            bx = BoxTab{};
            bx.g = h->g;
            for (int c = 0; c < 3; ++c) {
                bx.lo[c] = h->band_lo[c];
                bx.ext[c] = h->has_cond ? h->band_hi[c] - h->band_lo[c] + 1 : 0;
            }
            bx.x = h->ac;
            bx.y = h->bcpl;
            fin[i] = FinArgs{h->g.npad, A[i], h->ac, h->sj, h->sc, h->ctrl_d};
            b->nc_max = std::max(b->nc_max, h->nc);
            b->box_tpx = std::max(b->box_tpx, spmv_box_tpx(bx.ext));
            b->npad_max = std::max<int64_t>(b->npad_max, h->g.npad);
        }
        HIP_TRY(h0, hipMemcpyAsync(b->step_tab, stp.data(), ni * sizeof(StepArgs),
                                   hipMemcpyHostToDevice, b->st));
        HIP_TRY(h0, hipMemcpyAsync(b->upd_tab, upd.data(), ni * sizeof(UpdArgs),
                                   hipMemcpyHostToDevice, b->st));
        HIP_TRY(h0, hipMemcpyAsync(b->box_tab, box.data(), ni * sizeof(BoxTab),
                                   hipMemcpyHostToDevice, b->st));
        HIP_TRY(h0, hipMemcpyAsync(b->fin_tab, fin.data(), ni * sizeof(FinArgs),
                                   hipMemcpyHostToDevice, b->st));
        HIP_TRY(h0, hipStreamSynchronize(b->st));   // the host vectors go out of scope
    }
    b->slot_tpx = 1;
    for (int s = 0; s < 2; ++s) {
        const int seq = s == 0 ? EC_SEQ_SRC : EC_SEQ_CPL;
        b->tab[s].clear();
        std::vector<MdArgs> ms, m1, m2;
        std::vector<SmallArgs> ss, s1, s2, s3, s4;
        std::vector<LcArgs> ls, l1, l2;
        std::vector<SlotTab> sa;
        std::vector<RotArgs> ro;
        for (ec_problem *h : b->inst) {
            if (s == 0) b->tab[s].push_back(cg64_args(h, EC_SEQ_SRC, h->xs_d, &h->ctrl_d->scale,
                                                      h->sj, o, nullptr));
            else b->tab[s].push_back(cg64_args(h, EC_SEQ_CPL, h->bcpl, nullptr, h->sc, o, nullptr));
            if (!basis) continue;
            // the instance's start combination writes its residual sums here
            // (its pushes run after the solve's init)
            b->tab[s].back().start_part = h->part_md;
            seq_ensure(h, seq, meth, so->window, so->pod_kmax, so->pod_eps);
            seq_eta_ensure(h, seq, meth, spe_eta(h, o->precision));
            const CgArgs<double> &a = b->tab[s].back();
            const StartArgs st = seq_start_args(h, seq, meth, a.b, a.bscale, a.x, nullptr);
            ms.push_back(st.m);
            ss.push_back(st.s);
            ls.push_back(st.l);
            const PushArgs pa = seq_push_args(h, seq, meth, a.x, 0, false);
            m1.push_back(pa.m);
            m2.push_back(pa.m2);
            s1.push_back(pa.s1);
            s2.push_back(pa.s2);
            s3.push_back(pa.s3);
            s4.push_back(pa.s4);
            l1.push_back(pa.l1);
            l2.push_back(pa.l2);
            sa.push_back(SlotTab{h->g, h->ld, pa.sa});
            ro.push_back(pa.ro);
            b->slot_tpx = std::max(b->slot_tpx, spmv_slot_tpx(h->g));
        }
        HIP_TRY(h0, hipMemcpyAsync(b->tab_d[s], b->tab[s].data(),
                                   b->tab[s].size() * sizeof(CgArgs<double>),
                                   hipMemcpyHostToDevice, b->st));
        if (!basis) continue;
        const BasisTab &t = b->btab[s];
        auto up = [&](void *dst, const void *src, size_t bytes) -> int32_t {
            HIP_TRY(h0, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->st));
            return EC_OK;
        };
        int32_t rc = EC_OK;
        const size_t n = b->inst.size();
        if (!rc) rc = up(t.m_start, ms.data(), n * sizeof(MdArgs));
        if (!rc) rc = up(t.m, m1.data(), n * sizeof(MdArgs));
        if (!rc) rc = up(t.m2, m2.data(), n * sizeof(MdArgs));
        if (!rc) rc = up(t.s_start, ss.data(), n * sizeof(SmallArgs));
        if (!rc) rc = up(t.s1, s1.data(), n * sizeof(SmallArgs));
        if (!rc) rc = up(t.s2, s2.data(), n * sizeof(SmallArgs));
        if (!rc) rc = up(t.s3, s3.data(), n * sizeof(SmallArgs));
        if (!rc) rc = up(t.s4, s4.data(), n * sizeof(SmallArgs));
        if (!rc) rc = up(t.l_start, ls.data(), n * sizeof(LcArgs));
        if (!rc) rc = up(t.l1, l1.data(), n * sizeof(LcArgs));
        if (!rc) rc = up(t.l2, l2.data(), n * sizeof(LcArgs));
        if (!rc) rc = up(t.sa, sa.data(), n * sizeof(SlotTab));
        if (!rc) rc = up(t.ro, ro.data(), n * sizeof(RotArgs));
        if (rc) return rc;
        // the host vectors go out of scope: finish the copies first
        HIP_TRY(h0, hipStreamSynchronize(b->st));
    }
    HIP_TRY(h0, hipStreamSynchronize(b->st));
    return EC_OK;
}

static int32_t batch_solve(ec_batch_s *b, int s, const ec_step_opts *o)
{
    const int seq = s == 0 ? EC_SEQ_SRC : EC_SEQ_CPL;
    const int meth = o->start_method;
    const int n = (int)b->inst.size();
    const bool basis = meth == EC_SV_SPE || meth == EC_SV_POD;
    const BasisTab &t = b->btab[s];
    std::vector<int> modes(n);
    for (int i = 0; i < n; ++i) {
        ec_problem *h = b->inst[i];
        const CgArgs<double> &a = b->tab[s][i];
        int32_t rc = solve_prepare(h, seq, meth, o->window, o->pod_kmax, o->pod_eps, a.b, a.bscale,
                                   a.x, &o->solve, nullptr, &modes[i], false);
        if (rc) return rc;
    }
    if (basis) {                 // start vectors of all instances (eqs. 10, 14)
        multidot_tab(t.m_start, n, b->st);
        small_tab(t.s_start, n, meth == EC_SV_POD ? OP_POD_START : OP_SPE_START, b->st);
        lincomb_tab(t.l_start, n, false, b->st);
    }
    // PCG inits of all instances (same start method, so the same mode)
    if (modes[0] == START_X) {
        cg_init_batch(b->tab_d[s], b->inst_d, b->off_d, b->total_blocks, START_X, b->st);
        cg_init_batch(b->tab_d[s], b->inst_d, b->off_d, b->total_blocks, START_R2, b->st);
    } else {
        cg_init_batch(b->tab_d[s], b->inst_d, b->off_d, b->total_blocks, modes[0], b->st);
    }
    const int maxit = o->solve.maxit;
    int issued = 0;
    ec_problem *h0 = b->inst[0];
    if (capturing(h0)) {
        int budget = std::min(maxit, kGraphMaxIters);
        if (o->graph_iters[s] > 0) budget = std::min(budget, o->graph_iters[s]);
        // a budget below maxit: the last budgeted iteration and any further
        // ones of every instance run in one persistent launch over the block
        // map (same iteration bodies, so the same results as eager steps)
        const bool tail = budget < maxit && b->tail_blocks > 0;
        const int kernels = tail ? budget - 1 : budget;
        for (int it = 0; it < kernels; ++it)
            cg_iter_batch(b->tab_d[s], b->inst_d, b->off_d, b->total_blocks, it, b->one_tile,
                          b->st);
        if (tail) {
            hipError_t e = cg_tail_batch(b->tab_d[s], n, b->inst_d, b->off_d, b->total_blocks,
                                         kernels, b->tail_blocks, b->one_tile, b->st);
            if (e != hipSuccess)
                return fail(h0, EC_ERR_HIP, "batched tail launch: %s", hipGetErrorString(e));
        }
        issued = budget;
    } else {
        int chunk = 8;
        while (issued < maxit) {
            const int c = std::min(chunk, maxit - issued);
            for (int j = 0; j < c; ++j)
                cg_iter_batch(b->tab_d[s], b->inst_d, b->off_d, b->total_blocks, issued + j,
                              b->one_tile, b->st);
            issued += c;
            batch_done(b->tab_d[s], n, issued, b->flag_d, b->st);
            HIP_TRY(h0, hipMemcpyAsync(h0->pin + 20, b->flag_d, 4, hipMemcpyDeviceToHost, b->st));
            HIP_TRY(h0, hipStreamSynchronize(b->st));
            if (h0->pin[20]) break;
            chunk = std::min(2 * chunk, 256);
        }
    }
    cg_fin_batch(b->tab_d[s], n, issued, b->st);
    if (meth == EC_SV_POD) {     // histories of all instances
        spmv_slots_tab(t.sa, n, b->slot_tpx, b->st);
        multidot_tab(t.m, n, b->st);
        small_tab(t.s1, n, OP_POD_PUSH, b->st);
    } else if (meth == EC_SV_SPE) {
        multidot_tab(t.m, n, b->st);
        small_tab(t.s1, n, OP_SPE_PUSH1, b->st);
        lincomb_tab(t.l1, n, true, b->st);
        small_tab(t.s2, n, OP_SPE_PUSH2, b->st);
        lincomb_tab(t.l2, n, false, b->st);
        small_tab(t.s3, n, OP_SPE_PUSH3, b->st);
        spmv_slots_tab(t.sa, n, b->slot_tpx, b->st);
        multidot_tab(t.m2, n, b->st);
        small_tab(t.s4, n, OP_SPE_PUSH4, b->st);
        rotate_tab(t.ro, n, b->st);
    }
    return launch_check(h0, "batch solve");
}

static int32_t batch_step_impl(ec_batch_s *b, int64_t m, const double *dt, double *const *A,
                               const ec_step_opts *o)
{
    // the per-instance kernels of the step run from the device tables that
    // batch_tables filled for these dt and A (one launch each for the batch)
    (void)dt;
    (void)A;
    const int n = (int)b->inst.size();
    step_begin_tab(b->step_tab, n, m, b->st);
    int32_t rc;
    {
        Range r("source solve");
        rc = batch_solve(b, 0, o);
    }
    if (rc) return rc;
    {
        Range r("update");
        update_c_tab(b->upd_tab, n, b->nc_max, b->st);
        spmv_box_tab(b->box_tab, n, b->box_tpx, b->st);
    }
    {
        Range r("coupling solve");
        rc = batch_solve(b, 1, o);
    }
    if (rc) return rc;
    {
        Range r("finish state");
        finish_state_tab(b->fin_tab, n, b->npad_max, b->st);
    }
    return launch_check(b->inst[0], "batch step");
}

// pushes still due from launched graph steps of the instances (on their own
// streams, finished before the batch's work)
static int32_t batch_flush(ec_batch_s *b)
{
    for (ec_problem *h : b->inst)
        if (flush_pending(h)) HIP_TRY(h, hipStreamSynchronize(h->st));
    return EC_OK;
}

static int32_t batch_check(ec_batch_s *b, const double *dt, double *const *A,
                           const ec_step_opts *o)
{
    if (!b) return fail(nullptr, EC_ERR_ARG, "batch is NULL");
    if (!dt || !A || !o) return fail(nullptr, EC_ERR_ARG, "dt, A and opts are required");
    if (o->solve.precision != EC_PREC_FP64)
        return fail(nullptr, EC_ERR_ARG, "batched steps run FP64 solves");
    if (o->graph_iters[0] < 0 || o->graph_iters[1] < 0)
        return fail(nullptr, EC_ERR_ARG, "graph_iters must be >= 0");
    for (size_t i = 0; i < b->inst.size(); ++i) {
        if (b->inst[i]->mass_kind != EC_MASS_LUMPED)
            return fail(nullptr, EC_ERR_STATE, "instance %zu: batches use the lumped M_c", i);
        int32_t rc = check_step_args(b->inst[i], dt[i], A[i], o);
        if (rc) return fail(nullptr, rc, "instance %zu: %s", i, b->inst[i]->err.c_str());
    }
    return batch_flush(b);
}

extern "C" int32_t ec_batch_sizes(int32_t n, const ec_handle *handles, int64_t *bytes)
{
    if (n < 1 || !handles || !bytes) return fail(nullptr, EC_ERR_ARG, "need n >= 1, handles, bytes");
    std::vector<ec_problem *> hs(handles, handles + n);
    for (ec_problem *h : hs)
        if (!h || !h->bound) return fail(nullptr, EC_ERR_STATE, "every handle must be bound");
    *bytes = batch_layout(hs, nullptr, nullptr);
    return EC_OK;
}

extern "C" int32_t ec_batch_create(int32_t n, const ec_handle *handles, void *workspace,
                                   int64_t bytes, ec_batch *out)
{
    if (!out) return fail(nullptr, EC_ERR_ARG, "out is NULL");
    *out = nullptr;
    int64_t need = 0;
    int32_t rc = ec_batch_sizes(n, handles, &need);
    if (rc) return rc;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || bytes < need)
        return fail(nullptr, EC_ERR_ARG, "batch workspace: 256-byte aligned, >= %lld bytes",
                    (long long)need);
    std::vector<ec_problem *> hs(handles, handles + n);
    for (ec_problem *h : hs)
        if (h->st != hs[0]->st)
            return fail(nullptr, EC_ERR_ARG, "every handle must be bound to the same stream");
    ec_batch_s *b = new ec_batch_s();
    b->inst = hs;
    b->st = hs[0]->st;
    batch_layout(hs, (char *)workspace, b);
    b->tail_blocks = cg_tail_batch_blocks();
    rc = batch_apply_tiles(b, 1);
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return EC_OK;
}

extern "C" int32_t ec_batch_destroy(ec_batch b)
{
    delete b;
    return EC_OK;
}

extern "C" int32_t ec_batch_set_tiles(ec_batch b, int32_t tiles_per_block)
{
    if (!b || tiles_per_block < 1 || tiles_per_block > 64)
        return fail(nullptr, EC_ERR_ARG, "tiles_per_block must be 1..64");
    return batch_apply_tiles(b, tiles_per_block);
}

extern "C" int32_t ec_batch_step(ec_batch b, int64_t m, const double *dt, double *const *A,
                                 const ec_step_opts *opts)
{
    Range range("batch step");
    int32_t rc = batch_check(b, dt, A, opts);
    if (rc) return rc;
    rc = batch_tables(b, opts, dt, A);
    if (rc) return rc;
    return batch_step_impl(b, m, dt, A, opts);
}

extern "C" int32_t ec_batch_run(ec_batch b, int64_t m0, int64_t nsteps, const double *dt,
                                double *const *A, const ec_step_opts *opts)
{
    int32_t rc = batch_check(b, dt, A, opts);
    if (rc) return rc;
    if (nsteps < 0) return fail(nullptr, EC_ERR_ARG, "nsteps must be >= 0");
    rc = batch_tables(b, opts, dt, A);
    if (rc) return rc;
    for (int64_t s = 0; s < nsteps; ++s) {
        rc = batch_step_impl(b, m0 < 0 ? -1 : m0 + 1 + s, dt, A, opts);
        if (rc) return rc;
    }
    return EC_OK;
}

extern "C" int32_t ec_batch_graph_capture(ec_batch b, const double *dt, double *const *A,
                                          const ec_step_opts *opts, void **graph_exec)
{
    int32_t rc = batch_check(b, dt, A, opts);
    if (rc) return rc;
    if (!graph_exec) return fail(nullptr, EC_ERR_ARG, "graph_exec is NULL");
    for (ec_problem *h : b->inst)
        for (int s : {EC_SEQ_SRC, EC_SEQ_CPL}) {
            seq_ensure(h, s, opts->start_method, opts->window, opts->pod_kmax, opts->pod_eps);
            seq_eta_ensure(h, s, opts->start_method, spe_eta(h, opts->solve.precision));
        }
    rc = batch_tables(b, opts, dt, A);
    if (rc) return rc;
    ec_problem *h0 = b->inst[0];
    hipGraph_t graph = nullptr;
    HIP_TRY(h0, hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    rc = batch_step_impl(b, -1, dt, A, opts);
    hipError_t e = hipStreamEndCapture(b->st, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(nullptr, EC_ERR_HIP, "end capture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(nullptr, EC_ERR_HIP, "instantiate: %s", hipGetErrorString(e));
    e = hipGraphUpload(ex, b->st);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(ex);
        return fail(nullptr, EC_ERR_HIP, "graph upload: %s", hipGetErrorString(e));
    }
    *graph_exec = (void *)new GraphBox{ex, nullptr, -1};
    return EC_OK;
}

// Average duration of one batched PCG iteration (every instance active) for
// the current grids: zero-start solves of the sources into scratch vectors.
// Time of one batched iteration launch: with every solve active (maxit
// large), or with every solve finished (maxit 1: iteration 0 works, from
// iteration 1 on every block leaves after its checks).
constexpr double kBatchIdleWeight = 8.0;

static int32_t batch_time_iteration(ec_batch_s *b, double *us, bool idle = false)
{
    ec_solve_opts o{};
    o.rtol = 1e-300;
    o.maxit = idle ? 1 : 1 << 30;
    std::vector<CgArgs<double>> t;
    for (ec_problem *h : b->inst) {
        CgArgs<double> a = cg64_args(h, EC_SEQ_USER, h->xs_d, &h->ctrl_d->one, h->t4, &o, nullptr);
        a.ctrl = nullptr;
        t.push_back(a);
        cg64_init(h, a, START_ZERO);
    }
    ec_problem *h0 = b->inst[0];
    HIP_TRY(h0, hipMemcpyAsync(b->tab_d[0], t.data(), t.size() * sizeof(CgArgs<double>),
                               hipMemcpyHostToDevice, b->st));
    const int warm = 4, reps = 40;
    for (int it = 0; it < warm; ++it)
        cg_iter_batch(b->tab_d[0], b->inst_d, b->off_d, b->total_blocks, it, b->one_tile,
                      b->st);
    hipEvent_t e0, e1;
    HIP_TRY(h0, hipEventCreate(&e0));
    HIP_TRY(h0, hipEventCreate(&e1));
    HIP_TRY(h0, hipEventRecord(e0, b->st));
    for (int it = warm; it < warm + reps; ++it)
        cg_iter_batch(b->tab_d[0], b->inst_d, b->off_d, b->total_blocks, it, b->one_tile,
                      b->st);
    HIP_TRY(h0, hipEventRecord(e1, b->st));
    HIP_TRY(h0, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(h0, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us = 1e3 * ms / reps;
    return launch_check(h0, "batch timing");
}

static std::string batch_signature(const ec_batch_s *b)
{
    std::string sig;
    hipDeviceProp_t prop{};
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        sig += prop.gcnArchName;
    sig += ":n" + std::to_string(b->inst.size());
    for (const ec_problem *h : b->inst)
        sig += ":" + std::to_string(h->g.nx) + "x" + std::to_string(h->g.ny) + "x" +
               std::to_string(h->g.nz);
    return sig;
}

extern "C" int32_t ec_batch_autotune(ec_batch b, const char *cache_path, int32_t *tiles_per_block,
                                     double *us_per_iter)
{
    if (!b) return fail(nullptr, EC_ERR_ARG, "batch is NULL");
    const std::string sig = batch_signature(b);
    // a cached pick for this device and batch shape
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char line[8192];
            int best_f = 0;
            double best_us = 0.0;
            while (std::fgets(line, sizeof line, f)) {
                char key[8000];
                int ff = 0;
                double uu = 0.0;
                if (std::sscanf(line, "ec-batch-tiles %7999s %d %lf", key, &ff, &uu) == 3 &&
                    sig == key && ff >= 1 && ff <= 64) {
                    best_f = ff;
                    best_us = uu;
                }
            }
            std::fclose(f);
            if (best_f) {
                int32_t rc = batch_apply_tiles(b, best_f);
                if (rc) return rc;
                if (tiles_per_block) *tiles_per_block = best_f;
                if (us_per_iter) *us_per_iter = best_us;
                return EC_OK;
            }
        }
    }
    // a captured batch step issues several launches in which most solves
    // have already finished for each one in which they all work: the pick
    // minimises active + kBatchIdleWeight x idle launch time
    int best_f = 1;
    double best_us = 1e300, best_cost = 1e300;
    for (int f : {1, 2, 4, 8}) {
        int32_t rc = batch_apply_tiles(b, f);
        if (rc) return rc;
        double us = 0.0, idle = 0.0;
        rc = batch_time_iteration(b, &us);
        if (!rc) rc = batch_time_iteration(b, &idle, true);
        if (rc) return rc;
        const double cost = us + kBatchIdleWeight * idle;
        if (cost < best_cost) {
            best_cost = cost;
            best_us = us;
            best_f = f;
        }
    }
    int32_t rc = batch_apply_tiles(b, best_f);
    if (rc) return rc;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "ec-batch-tiles %s %d %.4f\n", sig.c_str(), best_f, best_us);
            std::fclose(f);
        }
    }
    if (tiles_per_block) *tiles_per_block = best_f;
    if (us_per_iter) *us_per_iter = best_us;
    return EC_OK;
}

extern "C" int32_t ec_graph_capture_step(ec_handle h, double dt, double *A,
                                         const ec_step_opts *opts, ec_solve_info *dev_info,
                                         void **graph_exec)
{
    NEED_BOUND(h);
    int32_t rc = check_step_args(h, dt, A, opts);
    if (rc) return rc;
    if (!graph_exec) return fail(h, EC_ERR_ARG, "graph_exec is NULL");
    if (opts->graph_iters[0] < 0 || opts->graph_iters[1] < 0)
        return fail(h, EC_ERR_ARG, "graph_iters must be >= 0");
    flush_pending(h);
    const bool fork = !opts->graph_serial && opts->solve.precision == EC_PREC_FP64 &&
                      opts->start_method == EC_SV_SPE;
    // configure the histories eagerly so that no reset is recorded
    for (int s : {EC_SEQ_SRC, EC_SEQ_CPL}) {
        seq_ensure(h, s, opts->start_method, opts->window, opts->pod_kmax, opts->pod_eps);
        seq_eta_ensure(h, s, opts->start_method, spe_eta(h, opts->solve.precision));
    }
    HIP_TRY(h, hipStreamSynchronize(h->st));
    hipGraph_t graph = nullptr;
    HIP_TRY(h, hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
    h->graph_iters[EC_SEQ_SRC] = opts->graph_iters[0];
    h->graph_iters[EC_SEQ_CPL] = opts->graph_iters[1];
    // the pushes on a branch of their own (`fork` above: SPE histories and
    // FP64 solves), except for a chain on request; FP32-refined solves and
    // POD histories measured slower forked (a forked step pushes each
    // sequence in launches of its own, and POD's pushes do not hide beside
    // its one-block eigen-solves)
    rc = step_impl(h, -1, dt, A, opts, dev_info, fork);
    h->graph_iters[EC_SEQ_SRC] = h->graph_iters[EC_SEQ_CPL] = 0;
    hipError_t e = hipStreamEndCapture(h->st, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(h, EC_ERR_HIP, "end capture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(h, EC_ERR_HIP, "instantiate: %s", hipGetErrorString(e));
    // upload now, so that the first launch does not pay for it
    e = hipGraphUpload(ex, h->st);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(ex);
        return fail(h, EC_ERR_HIP, "graph upload: %s", hipGetErrorString(e));
    }
    const int meth = opts->start_method;
    const bool due = fork;   // forked: this launch leaves its coupling push due
    *graph_exec = (void *)new GraphBox{ex, due ? h : nullptr, meth};
    return EC_OK;
}

extern "C" int32_t ec_graph_launch(void *graph_exec, void *hip_stream)
{
    if (!graph_exec) return fail(nullptr, EC_ERR_ARG, "graph_exec is NULL");
    GraphBox *g = (GraphBox *)graph_exec;
    Range range("graph launch");
    hipError_t e = hipGraphLaunch(g->ex, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, EC_ERR_HIP, "graph launch: %s", hipGetErrorString(e));
    if (g->h) g->h->pending_meth = g->meth;
    return EC_OK;
}

extern "C" int32_t ec_graph_destroy(void *graph_exec)
{
    if (graph_exec) {
        GraphBox *g = (GraphBox *)graph_exec;
        // a replay may still be running on the problem's stream
        if (g->h && g->h->bound) (void)hipStreamSynchronize(g->h->st);
        (void)hipGraphExecDestroy(g->ex);
        delete g;
    }
    return EC_OK;
}

extern "C" const char *ec_last_error(ec_handle h)
{
    return h ? h->err.c_str() : g_create_error.c_str();
}
