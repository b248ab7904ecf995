"""Consistent conductivity matrix and explicit Euler steps that invert it
(TEST INFRASTRUCTURE; only tests/, smoke() and bench.py's CPU leg use it).

The last paragraph of Sec. III notes that a non-diagonal M_c makes M_c^{-1}
in eq. (6) a further sequence of linear systems (the paper inverts M_c with
MAGMA, Sec. IV).  On the FIT grid the conductivity matrix is the lumped
(diagonal) one; its consistent counterpart is the mass matrix of the lowest-
order hexahedral edge elements:

* In a cell of sides h = (hx, hy, hz) and conductivity sigma the basis
  function of an edge of direction c is phi(u, v) / h_c times the unit vector
  of c, with (u, v) the two transverse coordinates and phi the bilinear hat of
  the transverse face that is 1 on that edge (so the line integral of the
  basis along its edge is 1, the FIT degree of freedom).
* M_ef = sigma / h_c^2 * h_c * integral of phi_e phi_f over the face
  = sigma h_a1 h_a2 / h_c * {1/9 (e = f), 1/18 (sharing a side), 1/36
  (diagonal)} for the four parallel edges of the cell, summed over cells.
* Row sums give sigma h_a1 h_a2 / (4 h_c) per cell: the lumped M_sigma.

Only conducting cells contribute, so M_c couples conducting edges only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .startvec import mgs_basis


def hat_integrals(n=4):
    """Integrals over the unit square of phi_0 phi_k for the bilinear hats at
    the corners (0,0), (1,0), (0,1), (1,1), by n-point Gauss quadrature."""
    xg, wg = np.polynomial.legendre.leggauss(n)
    xg, wg = 0.5 * (xg + 1.0), 0.5 * wg
    U, V = np.meshgrid(xg, xg, indexing="ij")
    W = np.outer(wg, wg)
    hats = [(1 - U) * (1 - V), U * (1 - V), (1 - U) * V, U * V]
    return [float((hats[0] * h * W).sum()) for h in hats]


def mass_matrix(P):
    """Consistent M_c (scipy CSR) on the conducting edges, in the order of
    np.flatnonzero(P.C), built cell by cell from the definition."""
    wl = P.wl
    nx, ny, nz = wl.n
    hh = [L / n for L, n in zip(wl.length, wl.n)]
    px, py = nx + 1, ny + 1
    S = px * py * (nz + 1)
    cslots = np.flatnonzero(P.C)
    pos = -np.ones(3 * S, np.int64)
    pos[cslots] = np.arange(len(cslots))
    sig = np.array([0.0] + [m.sigma for m in wl.materials])
    cm = np.asarray(wl.cell_mat).reshape(nz, ny, nx)
    I0 = hat_integrals()               # same corner, along u, along v, diagonal
    rows, cols, vals = [], [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                s = sig[cm[k, j, i]]
                if s == 0.0:
                    continue
                for c in range(3):
                    a1, a2 = (c + 1) % 3, (c + 2) % 3
                    scale = s * hh[a1] * hh[a2] / hh[c]
                    # the four edges of direction c of the cell: offsets
                    # (d1, d2) in {0,1}^2 along a1, a2
                    slots = []
                    for d2 in (0, 1):
                        for d1 in (0, 1):
                            node = [i, j, k]
                            node[a1] += d1
                            node[a2] += d2
                            slots.append(c * S + (node[2] * py + node[1]) * px + node[0])
                    for e in range(4):
                        for f in range(4):
                            rel = (e & 1) ^ (f & 1), (e >> 1) ^ (f >> 1)
                            w = I0[rel[0] + 2 * rel[1]]
                            rows.append(pos[slots[e]])
                            cols.append(pos[slots[f]])
                            vals.append(scale * w)
    assert min(rows) >= 0 and min(cols) >= 0, "a conducting cell edge outside C"
    n = len(cslots)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def spe_start_op(X, b, apply, dep_tol=1e-10):
    """x0 = U (U^T M U)^{-1} U^T b over the orthonormalised window X for the
    SPD operator `apply` (eq. 10 with M_c in place of K_n)."""
    U = mgs_basis(X, dep_tol)
    if not U:
        return np.zeros_like(b)
    Um = np.column_stack(U)
    MU = np.column_stack([apply(u) for u in U])
    return Um @ np.linalg.solve(Um.T @ MU, Um.T @ b)


def step(P, M, A, sc, m, dt, rtol=1e-12):
    """One explicit Euler step m of eqs. (6)-(7) (sign of eq. 5a) with
    a_c^m = a_c^{m-1} - dt M^{-1} g, M given on the conducting edges (sparse),
    the solves with K_n by the oracle's CG from zero.  Returns (A, sc)."""
    C, N = P.C, P.N
    sj, _, _, st = P.cg(P.source(m, dt), rtol=rtol)
    assert st == 0
    x = np.where(C, A, 0.0) + np.where(N, sj - sc, 0.0)
    g = P.apply(x, np.where(C, A, 0.0))[C]
    y = spla.spsolve(M.tocsc(), g)
    ac = np.zeros(P.n_pad)
    ac[C] = A[C] - dt * y
    sc_new, _, _, st = P.cg(P.kcnT(ac), rtol=rtol)
    assert st == 0
    out = np.where(C, ac, 0.0) + np.where(N, sj - sc_new, 0.0)
    return out, sc_new


def run(P, M, dt, nsteps, rtol=1e-12, A=None, sc=None, m0=0):
    """Steps m0+1 .. m0+nsteps of `step`; A and s_c start at rest unless given."""
    A = np.zeros(P.n_pad) if A is None else np.array(A, np.float64)
    sc = np.zeros(P.n_pad) if sc is None else np.array(sc, np.float64)
    for m in range(m0 + 1, m0 + nsteps + 1):
        A, sc = step(P, M, A, sc, m, dt, rtol)
    return A, sc
