"""Stability bound of the explicit Euler step and adaptive time steps
(TEST INFRASTRUCTURE; only tests/, smoke() and bench.py's CPU leg use it).

Eq. (8) bounds the step by dt <= 2 / lambda_max(M_c^{-1} K_S(a_c)), and the
paper estimates lambda_max by the power method (the sentence after eq. 8).
For the nonlinear reluctivity of eq. (1) two operators are of interest at a
state a:
* secant: M_c^{-1} (K_c(nu(a)) - S), the matrix of eq. (8) with nu frozen;
* Jacobian: M_c^{-1} (J_N(a) - S), J_N the derivative of
  N(a) = [C^T M_nu(a) C a]_C, so that one step linearised at a is
  I - dt M_c^{-1} (J_N(a) - S), S = K_cn K_n^+ K_cn^T.
The power method below runs on B = (X^T - S) M_c^{-1} with X = K_c(nu(a))
(symmetric) or X = J_N(a): B is the transpose of M_c^{-1} (X - S) (S is
symmetric), so it has the same eigenvalues; each iteration is one K_n^+
solve of the oracle's CG (zero start).  Norms are Euclidean on the
conducting edges; the estimate is ||B v|| for the unit iterate v.

Adaptive steps (the use the paper names for the estimate): the step of
m is dt_m = dt_max 2^-k with the smallest k >= 0 such that dt_m lambda <=
2 safety, lambda re-estimated at the state a^{m-1} every `every` steps.
"""
from __future__ import annotations

import numpy as np


def power(P, a, iters=200, rtol=1e-12, jacobian=True, seed=1):
    """Power-method estimate of |lambda|_max of M_c^{-1} (X(a) - S)."""
    C = P.C
    minv = np.where(C, 1.0 / np.where(C, P.msig, 1.0), 0.0)
    a = np.where(C, np.asarray(a, np.float64), 0.0)
    v = np.where(C, np.random.default_rng(seed).standard_normal(P.n_pad), 0.0)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = minv * v
        if jacobian:
            x = np.where(C, P.jnT(a, w), 0.0)
        else:
            x = np.where(C, P.apply(w, a), 0.0)          # K_c(nu(a)) w on C
        y = x - P.schur(w, rtol)
        lam = float(np.linalg.norm(y))
        v = y / lam
    return lam


def dense_spectrum(P, a, jacobian=True):
    """Eigenvalues of M_c^{-1} (X(a) - S) from dense matrices (tiny grids):
    X column by column from the oracle's J_N (or K(nu(a))), S from the dense
    Moore-Penrose pseudo-inverse of K_n."""
    from .dense import Dense
    C = P.C
    a = np.where(C, np.asarray(a, np.float64), 0.0)
    D = Dense(P)
    cs = D.c_slots
    X = np.zeros((len(cs), len(cs)))
    e = np.zeros(P.n_pad)
    for j, s in enumerate(cs):
        e[s] = 1.0
        X[:, j] = (P.jn(a, e) if jacobian else P.apply(e, a))[cs]
        e[s] = 0.0
    Kp, _ = D.pinv_kn()
    S = D.Kcn @ Kp @ D.Kcn.T
    return np.linalg.eigvals((X - S) / P.msig[cs][:, None])


def halving_dt(dt_max, lam, safety=0.5):
    """dt_max 2^-k, the smallest k >= 0 with dt lam <= 2 safety."""
    dt = float(dt_max)
    if not (lam > 0.0):
        return dt
    while dt * lam > 2.0 * safety:
        dt *= 0.5
    return dt


def adaptive_run(P, dt_max, nsteps, every, safety=0.5, power_iters=200, rtol=1e-12,
                 jacobian=True):
    """Explicit Euler steps 1..nsteps from rest with the adaptive rule; the
    source must be indexed by steps (DC or ramp).  Returns (A, dts, lambdas)."""
    assert P.wl.waveform in (0, 2), "adaptive reference: DC or ramp sources only"
    A = np.zeros(P.n_pad)
    sc = np.zeros(P.n_pad)
    dts, lams = [], []
    lam = 0.0
    for m in range(1, nsteps + 1):
        if (m - 1) % every == 0:
            lam = power(P, A, power_iters, rtol, jacobian)
            lams.append(lam)
        dt = halving_dt(dt_max, lam, safety)
        A, sc, *_ = P.run(dt, 1, rtol=rtol, A=A, sc=sc, m0=m - 1)
        dts.append(dt)
    return A, dts, lams
