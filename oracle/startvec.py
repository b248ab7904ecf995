"""Start vectors of Sec. III, written from the paper (TEST INFRASTRUCTURE).

* SPE, eq. (10): an orthonormal basis U of the span of previous solutions,
  built by modified Gram-Schmidt (with one reorthogonalisation pass) keeping
  only linearly independent columns, then the Galerkin projection
  x0 = U (U^T K_n U)^{-1} U^T b.  The right-hand side of eq. (10) is read as
  the current solve's right-hand side b of eq. (9).
* POD, eqs. (11)-(14): the SVD of the snapshot matrix X, truncation of the
  singular values by the threshold eps_POD = 1e-4 (keep sigma_i >= eps sigma_1,
  at most kmax modes), the relative information criterion of eq. (13), and
  the same Galerkin projection on the first k left singular vectors.
* Gauge penalty (reading of Sec. II, where grad-div regularisation is named as
  an alternative to the weak gauging of Krylov solvers): the projected matrix
  is U^T (K_n + eta D^T D) U, D the discrete divergence at the free nodes.
  K_n^+ b has zero divergence there, so the exact solution is unchanged; the
  penalty only stops the projection from amplifying the gradient (null-space)
  part that earlier solutions carry, which PCG never removes.  penalty = 0 is
  the projection of eq. (10) as printed.  POD keeps penalty = 0: its
  truncation (eq. 12) already drops the weak directions that carry that part.

K_n products come from the oracle's operator.  Everything else is numpy.
"""
from __future__ import annotations

import numpy as np

from .dense import divergence


def free_nodes(P):
    """Interior grid nodes that are not an end of any conducting edge."""
    nx, ny, nz = P.wl.n
    S = (nx + 1) * (ny + 1) * (nz + 1)
    k, r = np.divmod(np.arange(S), (nx + 1) * (ny + 1))
    j, i = np.divmod(r, nx + 1)
    free = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
    step = (1, nx + 1, (nx + 1) * (ny + 1))
    for c in range(3):
        tail = np.flatnonzero(P.C[c * S:(c + 1) * S])
        free[tail] = False
        free[tail + step[c]] = False
    return free


def gauge_rows(P, x, free=None):
    """D x: the divergence G^T x at the free nodes."""
    free = free_nodes(P) if free is None else free
    return divergence(P.wl.n, np.asarray(x, np.float64))[free]


def gauge_eta(P):
    """Penalty weight: half the mean K_n diagonal of a free edge, so that
    eta D^T D has the diagonal of K_n (2 nodes per edge)."""
    h = [L / n for L, n in zip(P.wl.length, P.wl.n)]
    d = [2.0 * P.wl.nu0 * (h[(c + 1) % 3] / (h[c] * h[(c + 2) % 3]) +
                           h[(c + 2) % 3] / (h[c] * h[(c + 1) % 3])) for c in range(3)]
    return 0.5 * sum(d) / 3.0


def mgs_basis(X, dep_tol=1e-10):
    """Orthonormal basis of span(X) (columns oldest first) by modified
    Gram-Schmidt, two passes; a column whose orthogonal remainder is below
    dep_tol times its own norm is dropped as linearly dependent."""
    U = []
    for x in X:
        v = np.array(x, dtype=np.float64)
        nx = np.linalg.norm(v)
        if nx == 0.0:
            continue
        for _ in range(2):
            for u in U:
                v -= (u @ v) * u
        nv = np.linalg.norm(v)
        if nv > dep_tol * nx:
            U.append(v / nv)
    return U


def galerkin(P, U, b, penalty=1.0):
    """x0 = U (U^T (K_n + eta D^T D) U)^{-1} U^T b for a list of basis vectors U,
    eta = penalty * gauge_eta(P)."""
    if len(U) == 0:
        return np.zeros_like(b)
    Um = np.column_stack(U)
    KU = np.column_stack([P.kn(u) for u in U])
    H = Um.T @ KU
    if penalty:
        free = free_nodes(P)
        DU = np.column_stack([gauge_rows(P, u, free) for u in U])
        H = H + penalty * gauge_eta(P) * (DU.T @ DU)
    y = np.linalg.solve(H, Um.T @ b)
    return Um @ y


def spe_start(P, X, b, dep_tol=1e-10, penalty=1.0):
    """SPE start vector (eq. 10) over the window X of previous solutions."""
    return galerkin(P, mgs_basis(X, dep_tol), b, penalty)


def pod_basis(X, eps=1e-4, kmax=None):
    """Left singular vectors kept by the POD truncation, and the eq. (13) value."""
    Xm = np.column_stack(X)
    Us, s, _ = np.linalg.svd(Xm, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return [], 0, 1.0, s
    k = int(np.count_nonzero(s >= eps * s[0]))
    if kmax is not None:
        k = min(k, kmax)
    info = float(s[:k].sum() / s.sum())
    return [Us[:, i] for i in range(k)], k, info, s


def pod_start(P, X, b, eps=1e-4, kmax=None, penalty=0.0):
    """POD start vector (eq. 14); returns (x0, k, information of eq. 13)."""
    U, k, info, _ = pod_basis(X, eps, kmax)
    return galerkin(P, U, b, penalty), k, info
