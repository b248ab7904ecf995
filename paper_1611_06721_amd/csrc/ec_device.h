// ec_device.h -- device helpers shared by the library's kernels: node
// decoding, edge classification, wave/block reductions and the curl-curl
// stencil of one grid node.
#pragma once
#include <hip/hip_runtime.h>

#include "ec_internal.h"

namespace ec {

// flat node index -> (i, j, k); exact for < 2^25 nodes (see the 1e-7 guard:
// a non-integer quotient is at least 1/(px*py) > 1e-7 away from the next one)
__device__ __forceinline__ void decode(const Geo &g, int64_t n, int &i, int &j, int &k)
{
    const int64_t pxy = (int64_t)g.px * g.py;
    k = (int)((double)n * (1.0 / (double)pxy) + 1e-7);
    const int64_t rem = n - (int64_t)k * pxy;
    j = (int)((double)rem * (1.0 / (double)g.px) + 1e-7);
    i = (int)(rem - (int64_t)j * g.px);
}

// 0 Dirichlet/padding, 1 conducting, 2 nonconducting (Sec. II dof split)
__device__ __forceinline__ int edge_cls(const Geo &g, int c, int i, int j, int k, int64_t n)
{
    if (c == 0) {
        if (i >= g.nx || j <= 0 || j >= g.ny || k <= 0 || k >= g.nz) return 0;
    } else if (c == 1) {
        if (j >= g.ny || i <= 0 || i >= g.nx || k <= 0 || k >= g.nz) return 0;
    } else {
        if (k >= g.nz || i <= 0 || i >= g.nx || j <= 0 || j >= g.ny) return 0;
    }
    if (!g.box) return g.cls[(int64_t)c * g.S + n];
    const int e0 = c == 0 ? 0 : 1, e1 = c == 1 ? 0 : 1, e2 = c == 2 ? 0 : 1;
    const bool inC = i >= g.clo[0] && i <= g.chi[0] + e0 && j >= g.clo[1] &&
                     j <= g.chi[1] + e1 && k >= g.clo[2] && k <= g.chi[2] + e2;
    return inC ? 1 : 2;
}

// v of the lane that the DPP control CTRL selects (both 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint2 u = __builtin_bit_cast(uint2, v);
    uint2 r;
    r.x = (unsigned)__builtin_amdgcn_mov_dpp((int)u.x, CTRL, 0xF, 0xF, false);
    r.y = (unsigned)__builtin_amdgcn_mov_dpp((int)u.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}

// Sum over the 64 lanes of a wave, the same value in every lane; every
// lane of the wave must be active.  Fixed order: pairs of lanes (lane ^ 1,
// then lane ^ 2) and the two halves of each 8-lane and 16-lane row by DPP
// (VALU, no LDS round trip), then row pairs and wave halves by the gfx950
// lane swaps (v_permlane16_swap / v_permlane32_swap).  Each step adds the
// same two operands in both partner lanes, so all lanes agree bitwise.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_f64<0x141>(v);   // row_half_mirror: the other quad of the 8 lanes
    v += dpp_f64<0x140>(v);   // row_mirror: the other 8 lanes of the row
    {
        const uint2 u = __builtin_bit_cast(uint2, v);
        const auto lo = __builtin_amdgcn_permlane16_swap(u.x, u.x, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(u.y, u.y, false, false);
        const double a = __builtin_bit_cast(double, make_uint2(lo[0], hi[0]));
        const double b = __builtin_bit_cast(double, make_uint2(lo[1], hi[1]));
        v = a + b;            // even row + odd row of each row pair
    }
    {
        const uint2 u = __builtin_bit_cast(uint2, v);
        const auto lo = __builtin_amdgcn_permlane32_swap(u.x, u.x, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(u.y, u.y, false, false);
        const double a = __builtin_bit_cast(double, make_uint2(lo[0], hi[0]));
        const double b = __builtin_bit_cast(double, make_uint2(lo[1], hi[1]));
        v = a + b;            // lower half + upper half
    }
    return v;
}

// Deterministic reduction of nvals <= NV values over the kMdBlocks block
// partials of a basis product (stored value-major: part[q * kMdBlocks + b])
// into the shared val[]: the first kMdBlocks threads (four waves) load one
// row each, every value is a fixed-order wave butterfly and then a fixed-
// order sum of the four waves.  All threads of the block (at least
// kMdBlocks) call it; the result does not depend on NV or nload.  The loads
// cover the first nload >= nvals values (a bound known before the count:
// they need not wait for the load that gives nvals; the partials buffer
// holds kMdStride values per block).
template <int NV>
__device__ __forceinline__ void reduce_rows(const double *part, int nload, int nvals, double *val)
{
    __shared__ double tmp[NV][4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < kMdBlocks) {
        double r[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) r[q] = q < nload ? part[(int64_t)q * kMdBlocks + tid] : 0.0;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            if (q < nvals) {
                const double s = wave_sum(r[q]);
                if (lane == 0) tmp[q][wv] = s;
            }
        }
    }
    __syncthreads();
    if (tid < nvals) val[tid] = ((tmp[tid][0] + tmp[tid][1]) + tmp[tid][2]) + tmp[tid][3];
    __syncthreads();
}

// Sum NV values over a block of blockDim.x <= 1024 threads; every thread
// gets the sums.  Fixed order: deterministic.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double lds[NV][16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[q][wv] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[q][w];
        v[q] = s;
    }
    __syncthreads();
}

// Deterministic sum of NV partial values over nb blocks (part[b*stride+q]),
// by the whole block; every thread gets the sums.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double *part, int nb, int stride,
                                                double (&out)[NV])
{
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q] += part[(int64_t)b * stride + q];
    }
    block_sum<NV>(out);
}

// K_air x at the three edges of node n: C^T M_nu0 C from the 24 edge values
// around the node.  ld(c, idx) returns the (possibly transformed) input at
// absolute index idx of direction block c.  The caller zeroes outputs on
// edges that are not nonconducting.  Out-of-range neighbours (only ever used
// by Dirichlet/padding outputs) are clamped into the array.
template <typename T, typename LD>
__device__ __forceinline__ void curlcurl_node(const Geo &g, int64_t n, LD ld, T &qx, T &qy,
                                              T &qz)
{
    const int64_t oi = 1, oj = g.px, ok = (int64_t)g.px * g.py;
    const int64_t S = g.S, S2 = 2 * g.S, last = 3 * g.S - 1;
    auto X = [&](int64_t o) {
        int64_t a = n + o;
        a = a < 0 ? 0 : a;
        return ld(0, a);
    };
    auto Y = [&](int64_t o) { return ld(1, S + n + o); };
    auto Z = [&](int64_t o) {
        int64_t a = S2 + n + o;
        a = a > last ? last : a;
        return ld(2, a);
    };
    const T x0 = X(0), x_kp = X(ok), x_km = X(-ok), x_im_kp = X(ok - oi), x_im = X(-oi),
            x_jp = X(oj), x_jm = X(-oj), x_im_jp = X(oj - oi);
    const T y0 = Y(0), y_kp = Y(ok), y_km = Y(-ok), y_jm = Y(-oj), y_jm_kp = Y(ok - oj),
            y_ip = Y(oi), y_ip_jm = Y(oi - oj), y_im = Y(-oi);
    const T z0 = Z(0), z_jp = Z(oj), z_jp_km = Z(oj - ok), z_km = Z(-ok), z_jm = Z(-oj),
            z_ip = Z(oi), z_ip_km = Z(oi - ok), z_im = Z(-oi);
    // face fluxes (right-handed circulation)
    const T Fx = y0 + z_jp - y_kp - z0;                // x-face (i,j,k)
    const T Fx_km = y_km + z_jp_km - y0 - z_km;        // x-face (i,j,k-1)
    const T Fx_jm = y_jm + z0 - y_jm_kp - z_jm;        // x-face (i,j-1,k)
    const T Fy = z0 + x_kp - z_ip - x0;                // y-face (i,j,k)
    const T Fy_km = z_km + x0 - z_ip_km - x_km;        // y-face (i,j,k-1)
    const T Fy_im = z_im + x_im_kp - z0 - x_im;        // y-face (i-1,j,k)
    const T Fz = x0 + y_ip - x_jp - y0;                // z-face (i,j,k)
    const T Fz_jm = x_jm + y_ip_jm - x0 - y_jm;        // z-face (i,j-1,k)
    const T Fz_im = x_im + y0 - x_im_jp - y_im;        // z-face (i-1,j,k)
    const T wx = (T)g.wx, wy = (T)g.wy, wz = (T)g.wz;
    qx = wz * (Fz - Fz_jm) - wy * (Fy - Fy_km);
    qy = wx * (Fx - Fx_km) - wz * (Fz - Fz_im);
    qz = wy * (Fy - Fy_im) - wx * (Fx - Fx_jm);
}

// Tile loop of a node kernel run by block bid of nb (nb % 8 == 0): blocks
// bid = 8*loc + xcd sweep the tiles of XCD slab xcd (contiguous k-planes stay
// in that XCD's L2; a launch places block b on XCD b % 8, so a grid slice
// starting at a multiple of 8 keeps the mapping).
template <typename F>
__device__ __forceinline__ void for_tiles_b(int tiles, int64_t S, int bid, int nb, F fn)
{
    const int xcd = bid & 7, loc = bid >> 3, nloc = nb >> 3;
    const int tpx = (tiles + 7) >> 3;
    for (int t = loc; t < tpx; t += nloc) {
        const int tile = xcd * tpx + t;
        if (tile >= tiles) break;
        const int64_t n = (int64_t)tile * kTile + threadIdx.x;
        if (n < S) fn(n);
    }
}

// the same over the whole launch
template <typename F>
__device__ __forceinline__ void for_tiles(int tiles, int64_t S, F fn)
{
    const int nb = gridDim.x, xcd = blockIdx.x & 7, loc = blockIdx.x >> 3, nloc = nb >> 3;
    const int tpx = (tiles + 7) >> 3;
    for (int t = loc; t < tpx; t += nloc) {
        const int tile = xcd * tpx + t;
        if (tile >= tiles) break;
        const int64_t n = (int64_t)tile * kTile + threadIdx.x;
        if (n < S) fn(n);
    }
}

// ------------------------------------------------ single-reduction PCG
// State entering kernel i from the reduced partials t = (gamma, delta, rho,
// bb) of the previous kernel and its record prev.  Same in every block.
__device__ __forceinline__ CgCtl cg_state(const CgCtl &prev, const double (&t)[4], int i,
                                          double rtol, int maxit, double &beta)
{
    CgCtl c = prev;
    beta = 0.0;
    if (prev.done) return c;
    const double gam = t[0], del = t[1], rho = t[2];
    double den;
    if (i == 0) {
        c.bb = t[3];
        c.tol2 = rtol * rtol * c.bb;
        c.rho0 = rho;
        den = del;
    } else {
        beta = gam / prev.gamma;
        den = del - beta * gam / prev.alpha;
    }
    c.gamma = gam;
    c.rho = rho;
    c.alpha = gam / den;
    c.it = i;
    c.status = EC_OK;
    if (!(rho == rho) || rho > 1e300) {
        c.done = 1;
        c.status = EC_ERR_NONFINITE;
    } else if (c.bb == 0.0 || rho <= c.tol2) {
        c.done = 1;
    } else if (i >= maxit) {
        c.done = 1;
        c.status = EC_ERR_NOT_CONVERGED;
    } else if (!(den > 0.0) || !(gam > 0.0)) {
        c.done = 1;
        c.status = EC_ERR_BREAKDOWN;
    }
    return c;
}

// This thread's share of the nb block partials of iteration it (strided
// loads, summed in the same order as reduce_partials).
__device__ __forceinline__ void part_load(const double *P, int nb, double (&t)[4])
{
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] = 0.0;
    // four strides' loads in flight before any is summed (one round trip for
    // up to 4 x blockDim blocks)
    for (int b0 = threadIdx.x; b0 < nb; b0 += 4 * (int)blockDim.x) {
        double v[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + u * (int)blockDim.x;
            if (b < nb) {
                const double2 *p2 = reinterpret_cast<const double2 *>(P + (int64_t)b * 4);
                const double2 lo = p2[0], hi = p2[1];
                v[u][0] = lo.x; v[u][1] = lo.y; v[u][2] = hi.x; v[u][3] = hi.y;
            } else {
                v[u][0] = v[u][1] = v[u][2] = v[u][3] = 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) t[q] += v[u][q];
    }
}

}  // namespace ec
