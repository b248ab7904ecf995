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

K_n products come from the oracle's operator.  Everything else is numpy.
"""
from __future__ import annotations

import numpy as np


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


def galerkin(P, U, b):
    """x0 = U (U^T K_n U)^{-1} U^T b for a list of basis vectors U."""
    if len(U) == 0:
        return np.zeros_like(b)
    Um = np.column_stack(U)
    KU = np.column_stack([P.kn(u) for u in U])
    H = Um.T @ KU
    y = np.linalg.solve(H, Um.T @ b)
    return Um @ y


def spe_start(P, X, b, dep_tol=1e-10):
    """SPE start vector (eq. 10) over the window X of previous solutions."""
    return galerkin(P, mgs_basis(X, dep_tol), b)


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


def pod_start(P, X, b, eps=1e-4, kmax=None):
    """POD start vector (eq. 14); returns (x0, k, information of eq. 13)."""
    U, k, info, _ = pod_basis(X, eps, kmax)
    return galerkin(P, U, b), k, info
