"""Implicit Euler with Newton's method, the reference the paper compares the
semi-explicit scheme with (Secs. I and IV) (TEST INFRASTRUCTURE; only tests/,
smoke() and bench.py's CPU leg use it).

One implicit Euler step of the DAE (3) solves, with a_n eliminated as in
eqs. (4)-(5b) (a_n = K_n^+ (j^m - K_cn^T a_c)), for the conducting unknowns a:
    F(a) = M_c (a - a_old) / dt + N(a) - S a + K_cn K_n^+ j^m = 0,
N(a) = [C^T M_nu(a) C a]_C, S = K_cn K_n^+ K_cn^T.  With s_j = K_n^+ j^m and
s_c = K_n^+ K_cn^T a this is F(a) = M_c (a - a_old)/dt + g(a), g the
conducting rows of K(nu(a)) applied to a (+) (s_j - s_c) (the g of eq. 6 at
the new state).  Newton: J(a) d = -F(a), J = M_c/dt + J_N(a) - S, a += d,
from a = a_old, until ||F(a)|| <= tol ||F(a_old)||; the linear systems by
GMRES (scipy) on the operator, every product through the oracle's J_N and
its CG for K_n^+.  Then a_n = s_j - s_c(a).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def residual(P, a, a_old, sj, dt, rtol=1e-12):
    """(F(a) on C (compact), s_c(a)) for the padded conducting vectors a, a_old."""
    C, N = P.C, P.N
    sc, _, _, st = P.cg(P.kcnT(np.where(C, a, 0.0)), rtol=rtol)
    assert st == 0
    x = np.where(C, a, 0.0) + np.where(N, sj - sc, 0.0)
    g = P.apply(x, np.where(C, a, 0.0))[C]
    F = P.msig[C] * (a[C] - a_old[C]) / dt + g
    return F, sc


def jacobian_op(P, a, dt, rtol=1e-12):
    """The Newton matrix J(a) = M_c/dt + J_N(a) - S as a LinearOperator on
    compact conducting vectors."""
    C = P.C
    n = int(C.sum())
    mc = P.msig[C]

    def mv(v):
        x = np.zeros(P.n_pad)
        x[C] = v
        return mc * v / dt + P.jn(a, x)[C] - P.schur(x, rtol)[C]
    return spla.LinearOperator((n, n), matvec=mv, dtype=np.float64)


def step(P, A_old, m, dt, tol=1e-10, rtol=1e-12, gmres_rtol=1e-12, maxnewton=20):
    """Implicit Euler step m from the state A_old; returns (A, newton iterations,
    the residual norms ||F|| per iteration)."""
    C, N = P.C, P.N
    sj, _, _, st = P.cg(P.source(m, dt), rtol=rtol)
    assert st == 0
    a_old = np.where(C, A_old, 0.0)
    a = a_old.copy()
    norms = []
    F, sc = residual(P, a, a_old, sj, dt, rtol)
    f0 = np.linalg.norm(F)
    norms.append(f0)
    it = 0
    while f0 > 0.0 and norms[-1] > tol * f0 and it < maxnewton:
        J = jacobian_op(P, a, dt, rtol)
        d, info = spla.gmres(J, -F, rtol=gmres_rtol, atol=0.0, restart=60, maxiter=2000)
        assert info == 0
        a[C] += d
        F, sc = residual(P, a, a_old, sj, dt, rtol)
        norms.append(np.linalg.norm(F))
        it += 1
    A = np.where(C, a, 0.0) + np.where(N, sj - sc, 0.0)
    return A, it, norms


def run(P, dt, nsteps, A=None, m0=0, **kw):
    """Implicit Euler steps m0+1..m0+nsteps; returns (A, newton iterations per step)."""
    A = np.zeros(P.n_pad) if A is None else np.array(A, np.float64)
    its = []
    for m in range(m0 + 1, m0 + nsteps + 1):
        A, it, _ = step(P, A, m, dt, **kw)
        its.append(it)
    return A, its
