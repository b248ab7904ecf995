"""Discrete adjoint of the explicit Euler time loop (TEST INFRASTRUCTURE).

The time loop of eqs. (6)-(7) (sign of eq. 5a) advances the conducting
unknowns by
    a^m = F^m(a^{m-1}) = a^{m-1} - dt M_c^{-1} [ N(a^{m-1}) - S a^{m-1} + K_cn K_n^+ j^m ],
with N(a) = [C^T M_nu(a) C a]_C and S = K_cn K_n^+ K_cn^T (the step solves
K_n^+ K_cn^T a^{m-1} for s_c, so K_cn s_c = S a^{m-1}).  The loss is the
Joule loss of the conductor, sum_m dt sigma |da/dt|^2 integrated over space,
in the discrete form
    L = sum_{m=1}^{M} (1/dt) d_m^T M_c d_m,   d_m = a^m - a^{m-1}.
With mu_m = dL/da^m (through every later step):
    mu_M = (2/dt) M_c d_M,
    mu_m = (2/dt) M_c (d_m - d_{m+1}) + mu_{m+1} - dt [J_N(a^m)^T - S] M_c^{-1} mu_{m+1},
and, with M_c = M_sigma depending on sigma through dM_c/dsigma = Phi,
    dL/dsigma = sum_m [ (1/dt) d_m^T Phi d_m - mu_m^T M_c^{-1} Phi d_m ],
    dL/dk1    = -dt sum_m mu_m^T M_c^{-1} dN/dk1(a^{m-1}).
Every step of the forward run comes from the oracle's own time loop
(zero-start CG), every product from its operators.
"""
from __future__ import annotations

import numpy as np


def forward_states(P, dt, nsteps, rtol=1e-12, A0=None, m0=0):
    """a^0 .. a^M (full padded arrays; a^0 = A0 or 0) from the oracle's time loop."""
    A = np.zeros(P.n_pad) if A0 is None else np.array(A0, np.float64)
    sc = None
    if A0 is not None:
        sc, _, _, st = P.cg(P.kcnT(np.where(P.C, A, 0.0)), rtol=rtol)
        if st:
            raise RuntimeError("oracle CG failed")
    _, _, rec, _, _ = P.run(dt, nsteps, rtol=rtol, A=A, sc=sc, m0=m0, rec_every=1)
    return [np.where(P.C, A, 0.0)] + [np.where(P.C, r, 0.0) for r in rec]


def joule_loss(P, dt, states):
    mc = np.where(P.C, P.msig, 0.0)
    return sum(float(((b - a) * mc * (b - a)).sum()) / dt for a, b in zip(states[:-1], states[1:]))


def adjoint(P, dt, states, mat=1, rtol=1e-12):
    """(L, dL/dsigma, dL/dk1, mu) for the trajectory `states` (a^0..a^M)."""
    C = P.C
    mc = np.where(C, P.msig, 0.0)
    inv = np.where(C, 1.0 / np.where(C, P.msig, 1.0), 0.0)
    M = len(states) - 1
    d = [None] + [states[m] - states[m - 1] for m in range(1, M + 1)]
    mu = [None] * (M + 1)
    mu[M] = (2.0 / dt) * mc * d[M]
    for m in range(M - 1, 0, -1):
        w = inv * mu[m + 1]
        mu[m] = ((2.0 / dt) * mc * (d[m] - d[m + 1]) + mu[m + 1]
                 - dt * (P.jnT(states[m], w) - P.schur(w, rtol)))
    phi = P.dmsig(mat)
    loss = sum(float((d[m] * mc * d[m]).sum()) / dt for m in range(1, M + 1))
    g_sig = sum(float((d[m] * phi * d[m]).sum()) / dt - float((mu[m] * inv * phi * d[m]).sum())
                for m in range(1, M + 1))
    g_k1 = -dt * sum(float((mu[m] * inv * P.dn_dk1(states[m - 1], mat)).sum())
                     for m in range(1, M + 1))
    return loss, g_sig, g_k1, mu
