"""Pins of the consistent conductivity matrix and of explicit Euler with
M_c^{-1} as solves (oracle/mass.py): the hat integrals, row sums equal to
the lumped FIT M_sigma, symmetry and the spectrum bounds of the tensor-hat
mass, the stepper against the C oracle for the lumped matrix, and the
closed-form decay of a generalized eigenmode of (K_S, M_c)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from tests.conftest import small_workload
from tests.test_oracle_pins import _state_from_ac, cube


def test_hat_integrals():
    from oracle.mass import hat_integrals
    got = hat_integrals()
    assert np.allclose(got, [1 / 9, 1 / 18, 1 / 18, 1 / 36], rtol=1e-14, atol=0)


@pytest.mark.parametrize("wl_fn", [lambda: cube(6), lambda: small_workload(),
                                   lambda: synth.nonlinear(8, ramp_steps=10)])
def test_mass_rows_lump_to_fit(oracle_mod, wl_fn):
    """Row sums are the lumped FIT conductivity (also on non-cubic cells);
    M is symmetric positive definite, and lumped^-1 M has its spectrum in
    [1/9, 1] (the 2D tensor of the 1D consistent/lumped range [1/3, 1])."""
    from oracle.mass import mass_matrix
    P = oracle_mod.Problem(wl_fn())
    M = mass_matrix(P)
    lump = P.msig[P.C]
    assert np.allclose(np.asarray(M.sum(axis=1)).ravel(), lump, rtol=1e-13, atol=0)
    D = M.toarray()
    assert np.array_equal(D, D.T)
    d = 1.0 / np.sqrt(lump)
    ev = np.linalg.eigvalsh(d[:, None] * D * d[None, :])
    assert ev.min() >= 1 / 9 - 1e-12 and ev.max() <= 1.0 + 1e-12
    assert ev.min() < 0.5                          # really not the lumped matrix


def test_stepper_with_lumped_matrix_equals_c_oracle(oracle_mod):
    """The Python stepper of eq. (6)-(7) with the lumped M_c reproduces the C
    oracle's time loop (two independent implementations of the step)."""
    from oracle import mass
    wl = synth.linear_c1(12)
    P = oracle_mod.Problem(wl)
    dt = 0.9 * 2 / P.power(iters=40)
    Ml = sp.diags(P.msig[P.C]).tocsr()
    A, _ = mass.run(P, Ml, dt, 12)
    Ao, *_ = P.run(dt, 12, rtol=1e-12)
    assert np.linalg.norm(A - Ao) <= 1e-11 * np.linalg.norm(Ao)


def test_closed_form_decay_consistent_mass(oracle_mod):
    """j = 0, a_c^0 = v with K_S v = lambda M v (M consistent): the steps give
    a_c^m = (1 - dt lambda)^m v (eq. 6 with M_c^{-1} applied exactly)."""
    from oracle import mass
    from oracle.dense import Dense
    wl = cube(6)
    wl.amp = 0.0
    P = oracle_mod.Problem(wl)
    M = mass.mass_matrix(P)
    D = Dense(P)
    assert np.array_equal(D.c_slots, np.flatnonzero(P.C))
    KS = D.schur()
    Md = M.toarray()
    L = np.linalg.cholesky(Md)
    Li = np.linalg.inv(L)
    lam, Y = np.linalg.eigh(Li @ KS @ Li.T)
    dt = 0.9 * 2 / lam.max()
    for idx in (0, len(lam) - 1):
        v = Li.T @ Y[:, idx]
        ac = np.zeros(P.n_pad)
        ac[P.C] = v / np.abs(v).max()
        A, sc = _state_from_ac(P, ac)
        for m in range(1, 6):
            A, sc = mass.step(P, M, A, sc, m, dt)
            want = (1 - dt * lam[idx]) ** m * ac[P.C]
            assert np.linalg.norm(A[P.C] - want) <= 1e-10 * np.linalg.norm(ac[P.C])


def test_spe_start_with_mass_operator(oracle_mod):
    """The Galerkin start of eq. (10) with M_c: exact when b = M x for x in
    the window's span, and M-orthogonal residual otherwise."""
    from oracle.mass import mass_matrix, spe_start_op
    P = oracle_mod.Problem(synth.nonlinear(8, ramp_steps=10))
    M = mass_matrix(P)
    rng = np.random.default_rng(3)
    X = [rng.standard_normal(M.shape[0]) for _ in range(5)]
    x = 0.3 * X[1] - 2.0 * X[4]
    x0 = spe_start_op(X, M @ x, lambda u: M @ u)
    assert np.linalg.norm(x0 - x) <= 1e-10 * np.linalg.norm(x)
    b = rng.standard_normal(M.shape[0])
    x0 = spe_start_op(X, b, lambda u: M @ u)
    r = b - M @ x0
    for u in X:
        assert abs(u @ r) <= 1e-10 * np.linalg.norm(u) * np.linalg.norm(b)
