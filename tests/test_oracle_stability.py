"""Pins of the stability-bound oracle (oracle/stability.py): the power
method against dense eigenvalues (secant operator of eq. 8 and the Jacobian
one at a saturated state), the halving rule, and adaptive steps that stay
bounded where a fixed step beyond eq. (8) grows."""
import numpy as np
import pytest

import synth
from tests.test_oracle_adjoint import iron8, saturated_state
from tests.test_oracle_pins import cube


def test_power_secant_equals_dense_eq8(oracle_mod):
    """Linear case: the secant operator is M_c^{-1} K_S of eq. (8); the power
    estimate equals the largest generalized eigenvalue of (K_S, M_c)."""
    from oracle.dense import Dense
    from oracle.stability import dense_spectrum, power
    wl = cube(6)
    P = oracle_mod.Problem(wl)
    lam_dense = Dense(P).gen_eig()[0].max()
    ev = dense_spectrum(P, np.zeros(P.n_pad), jacobian=False)
    assert np.abs(ev).max() == pytest.approx(lam_dense, rel=1e-10)
    assert power(P, np.zeros(P.n_pad), iters=400, jacobian=False) == \
        pytest.approx(lam_dense, rel=1e-6)
    # linear: the Jacobian operator is the same matrix
    assert power(P, np.zeros(P.n_pad), iters=400, jacobian=True) == \
        pytest.approx(lam_dense, rel=1e-6)


def test_power_jacobian_equals_dense_saturated(oracle_mod):
    """Brauer iron near 1 T: |lambda|_max of M_c^{-1} (J_N(a) - S) from the
    power method equals the dense spectrum's; the dominant eigenvalue is real,
    and the Jacobian bound is tighter than the secant one (nu' > 0)."""
    from oracle.stability import dense_spectrum, power
    P = oracle_mod.Problem(iron8())
    a = saturated_state(P)
    ev = dense_spectrum(P, a, jacobian=True)
    top = ev[np.argmax(np.abs(ev))]
    assert abs(top.imag) <= 1e-9 * abs(top)
    lam = power(P, a, iters=600, jacobian=True)
    assert lam == pytest.approx(abs(top), rel=1e-6)
    ev_s = dense_spectrum(P, a, jacobian=False)
    lam_s = power(P, a, iters=600, jacobian=False)
    assert lam_s == pytest.approx(np.abs(ev_s).max(), rel=1e-6)
    assert lam > lam_s


def test_halving_rule():
    from oracle.stability import halving_dt
    assert halving_dt(1.0, 0.9, 0.5) == 1.0
    assert halving_dt(1.0, 1.1, 0.5) == 0.5
    assert halving_dt(1.0, 4.0, 0.5) == 0.25
    assert halving_dt(1.0, 4.0000001, 0.5) == 0.125
    assert halving_dt(3.0, 0.0, 0.5) == 3.0


def test_adaptive_steps_stay_bounded(oracle_mod):
    """A dt three times the bound of eq. (8) at rest: fixed steps grow by
    orders of magnitude, adaptive steps (halving rule, bound re-estimated
    every 5 steps) stay bounded and every dt meets the rule."""
    from oracle.stability import adaptive_run, halving_dt, power
    wl = synth.nonlinear(8, ramp_steps=10, J0=4.0e7)
    P = oracle_mod.Problem(wl)
    lam0 = power(P, np.zeros(P.n_pad), iters=300, jacobian=True)
    dt_max = 3.0 * 2.0 / lam0
    A_ad, dts, lams = adaptive_run(P, dt_max, 30, 5, safety=0.5, power_iters=300)
    A_fx, *_ = P.run(dt_max, 30, rtol=1e-12)
    A_ref, *_ = P.run(0.5 * 2.0 / lam0, 30, rtol=1e-12)
    nf = np.linalg.norm(A_fx)                      # overflows (Brauer exp) or grows
    assert not np.isfinite(nf) or nf > 1e3 * np.linalg.norm(A_ref)
    assert np.linalg.norm(A_ad) < 10.0 * np.linalg.norm(A_ref)
    for m, dt in enumerate(dts):
        assert dt == halving_dt(dt_max, lams[m // 5], 0.5)
        assert dt * lams[m // 5] <= 1.0
