"""Pins of the implicit Euler / Newton reference (oracle/implicit.py): one
Newton step solves the linear case exactly (the dense Schur system), a
generalized eigenmode decays by (1 + dt lambda)^-m far beyond the explicit
bound of eq. (8), and Newton converges quadratically on saturated iron."""
import numpy as np
import pytest

import synth
from tests.test_oracle_adjoint import iron8
from tests.test_oracle_pins import _state_from_ac, cube


def test_linear_step_equals_dense_schur_solve(oracle_mod):
    from oracle import implicit
    from oracle.dense import Dense
    wl = cube(6)
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    lmax = D.gen_eig()[0].max()
    dt = 20 * 2 / lmax
    rng = np.random.default_rng(4)
    A_old = np.zeros(P.n_pad)
    A_old[P.C] = rng.standard_normal(int(P.C.sum()))
    m = 3
    A, its, norms = implicit.step(P, A_old, m, dt)
    assert its == 1
    Kp, _ = D.pinv_kn()
    j = P.source(m, dt)[D.n_slots]
    mc = D.Mc
    rhs = mc * A_old[D.c_slots] / dt - D.Kcn @ (Kp @ j)
    a = np.linalg.solve(np.diag(mc / dt) + D.schur(), rhs)
    assert np.linalg.norm(A[D.c_slots] - a) <= 1e-10 * np.linalg.norm(a)
    an = Kp @ (j - D.Kcn.T @ a)
    assert np.linalg.norm(A[D.n_slots] - an) <= 1e-9 * np.linalg.norm(an)


def test_eigenmode_decays_beyond_the_explicit_bound(oracle_mod):
    """j = 0, a^0 = v (K_S v = lambda M_c v): a^m = (1 + dt lambda)^-m v for
    dt 50 times the explicit bound (implicit Euler is unconditionally stable)."""
    from oracle import implicit
    from oracle.dense import Dense
    wl = cube(6)
    wl.amp = 0.0
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    lam, V = D.gen_eig()
    dt = 50 * 2 / lam.max()
    for idx in (0, len(lam) - 1):
        ac = np.zeros(P.n_pad)
        ac[D.c_slots] = V[:, idx] / np.abs(V[:, idx]).max()
        A, _ = _state_from_ac(P, ac)
        for m in range(1, 4):
            A, _, _ = implicit.step(P, A, m, dt)
            want = (1 + dt * lam[idx]) ** -m * ac[D.c_slots]
            assert np.linalg.norm(A[D.c_slots] - want) <= 1e-9 * np.linalg.norm(ac[D.c_slots])


def test_newton_quadratic_on_saturated_iron(oracle_mod):
    from oracle import implicit
    from tests.test_oracle_adjoint import saturated_state
    P = oracle_mod.Problem(iron8())
    a0 = saturated_state(P, scale=0.6)
    dt = 20 * 2 / P.power(iters=60)
    A, its, norms = implicit.step(P, a0, 5, dt, tol=1e-13)
    assert 3 <= its <= 10
    assert norms[-1] <= 1e-13 * norms[0]
    # asymptotically quadratic: ||F_k+1|| ~ K ||F_k||^2 with the same K for
    # the last two iterations (the Jacobian is exact)
    k2 = norms[-1] / norms[-2] ** 2
    k1 = norms[-2] / norms[-3] ** 2
    assert k2 <= 10 * k1
    assert norms[-1] / norms[-2] < 1e-5
