"""Dense matrices of tiny grids, for pinning the oracle (TEST INFRASTRUCTURE).

The matrices are read off the oracle's operators column by column, then
checked against facts the mathematics fixes: symmetry, the discrete gradient
in the null space (curl grad = 0), the nullity of the nonconducting block, the
Moore-Penrose pseudo-inverse from an eigendecomposition (the pseudo-inverse of
eq. (4)), and the generalized eigenpairs of the Schur complement that give the
closed-form decay of explicit Euler and the bound of eq. (8).
"""
from __future__ import annotations

import numpy as np


class Dense:
    def __init__(self, P, state=None):
        """Dense K on the non-Dirichlet edges of oracle problem P."""
        self.P = P
        self.idx = np.flatnonzero(~P.D)           # interior edge slots
        self.ic = np.flatnonzero(P.C[self.idx])   # positions of C inside idx
        self.inn = np.flatnonzero(P.N[self.idx])  # positions of N inside idx
        n = len(self.idx)
        K = np.zeros((n, n))
        st = np.zeros(P.n_pad) if state is None else state
        e = np.zeros(P.n_pad)
        for col, slot in enumerate(self.idx):
            e[slot] = 1.0
            K[:, col] = P.apply(e, st)[self.idx]
            e[slot] = 0.0
        self.K = K
        self.Kc = K[np.ix_(self.ic, self.ic)]
        self.Kcn = K[np.ix_(self.ic, self.inn)]
        self.Kn = K[np.ix_(self.inn, self.inn)]
        self.Mc = P.msig[self.idx][self.ic]

    # slots of the padded array for the C and N blocks
    @property
    def c_slots(self):
        return self.idx[self.ic]

    @property
    def n_slots(self):
        return self.idx[self.inn]

    def pinv_kn(self, rel=1e-9):
        """Moore-Penrose pseudo-inverse of K_n from its eigendecomposition."""
        w, V = np.linalg.eigh(self.Kn)
        keep = w > rel * w.max()
        return (V[:, keep] / w[keep]) @ V[:, keep].T, V[:, ~keep]

    def schur(self):
        """K_S = K_c - K_cn K_n^+ K_cn^T (eq. 4), dense."""
        Kp, _ = self.pinv_kn()
        return self.Kc - self.Kcn @ Kp @ self.Kcn.T

    def gen_eig(self):
        """Generalized eigenpairs (lambda_i, v_i) of K_S v = lambda M_c v."""
        KS = self.schur()
        d = 1.0 / np.sqrt(self.Mc)
        w, Y = np.linalg.eigh(d[:, None] * KS * d[None, :])
        return w, d[:, None] * Y


def gradient(n, phi):
    """Discrete gradient G phi of node potentials (the definition of G):
    the x-edge (i,j,k) gets phi(i+1,j,k) - phi(i,j,k), likewise y and z."""
    nx, ny, nz = n
    ph = phi.reshape(nz + 1, ny + 1, nx + 1)
    S = (nx + 1) * (ny + 1) * (nz + 1)
    g = np.zeros(3 * S)
    gx = np.zeros((nz + 1, ny + 1, nx + 1))
    gy = np.zeros_like(gx)
    gz = np.zeros_like(gx)
    gx[:, :, :nx] = ph[:, :, 1:] - ph[:, :, :nx]
    gy[:, :ny, :] = ph[:, 1:, :] - ph[:, :ny, :]
    gz[:nz, :, :] = ph[1:, :, :] - ph[:nz, :, :]
    g[:S] = gx.ravel()
    g[S:2 * S] = gy.ravel()
    g[2 * S:] = gz.ravel()
    return g


def divergence(n, j):
    """G^T j for an edge array j (the transpose of `gradient`); zero for a
    discretely divergence-free current."""
    nx, ny, nz = n
    S = (nx + 1) * (ny + 1) * (nz + 1)
    jx = j[:S].reshape(nz + 1, ny + 1, nx + 1)
    jy = j[S:2 * S].reshape(nz + 1, ny + 1, nx + 1)
    jz = j[2 * S:].reshape(nz + 1, ny + 1, nx + 1)
    d = np.zeros((nz + 1, ny + 1, nx + 1))
    d[:, :, 1:] += jx[:, :, :nx]
    d[:, :, :nx] -= jx[:, :, :nx]
    d[:, 1:, :] += jy[:, :ny, :]
    d[:, :ny, :] -= jy[:, :ny, :]
    d[1:, :, :] += jz[:nz, :, :]
    d[:nz, :, :] -= jz[:nz, :, :]
    return d.ravel()
