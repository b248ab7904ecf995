"""Pins of the adjoint oracle (oracle/adjoint.py and the J_N / dN/dk1 / dM/dsigma
primitives of the C oracle): central differences of the forward operators,
dot-product tests of the written-out transposes, exact linearity in k1, the
central difference of the whole loss in sigma and k1, and the closed-form
Joule loss of a decaying generalised eigenmode."""
import copy

import numpy as np
import pytest

import synth
from tests.test_oracle_pins import _state_from_ac, cube


def iron8(J0=4.0e7, k1=None, sigma=2.0e6):
    """8^3 grid, Brauer iron 2^3 cells, coil ramped over 10 steps."""
    k = synth.BRAUER if k1 is None else (k1, synth.BRAUER[1], synth.BRAUER[2])
    return synth.nonlinear(8, ramp_steps=10, J0=J0, sigma=sigma, brauer=k)


def with_material(wl, **kw):
    w = copy.deepcopy(wl)
    m = w.materials[0]
    w.materials = [synth.Material(kw.get("sigma", m.sigma), kw.get("k1", m.k1), m.k2, m.k3)]
    return w


def saturated_state(P, scale=0.4):
    """A random conducting-edge state with |B| of order 1 T in the iron."""
    a = synth.random_vector(P.n_pad, P.C, 11)
    h = min(P.wl.length[i] / P.wl.n[i] for i in range(3))
    return a * scale * h * h / np.abs(a).max()


def test_jn_matches_central_difference(oracle_mod):
    P = oracle_mod.Problem(iron8())
    a = saturated_state(P)
    B = P.cell_B(a)[P.wl.cell_mat.astype(bool)]
    assert np.sqrt((B ** 2).sum(1)).max() > 0.5        # the nonlinearity matters
    for seed in (1, 2):
        v = synth.random_vector(P.n_pad, P.C, 20 + seed) * np.abs(a).max()
        eps = 1e-5
        fd = (P.n_c(a + eps * v) - P.n_c(a - eps * v)) / (2 * eps)
        jv = P.jn(a, v)
        assert np.linalg.norm(jv - fd) <= 1e-7 * np.linalg.norm(jv)
        assert not jv[~P.C].any()


def test_jn_transpose_dot_product(oracle_mod):
    P = oracle_mod.Problem(iron8())
    a = saturated_state(P)
    for seed in (3, 4, 5):
        v = synth.random_vector(P.n_pad, P.C, seed)
        lam = synth.random_vector(P.n_pad, P.C, 30 + seed)
        lhs = lam @ P.jn(a, v)
        rhs = P.jnT(a, lam) @ v
        assert lhs == pytest.approx(rhs, rel=1e-12)
    # J_N is not symmetric under the face-averaged reluctivity
    v = synth.random_vector(P.n_pad, P.C, 3)
    assert np.linalg.norm(P.jn(a, v) - P.jnT(a, v)) > 1e-6 * np.linalg.norm(P.jn(a, v))


def test_jn_linear_material_is_kc(oracle_mod):
    """k1 = 0: N(a) is linear, J_N = K_c."""
    P = oracle_mod.Problem(cube(8))
    a = synth.random_vector(P.n_pad, P.C, 7)
    v = synth.random_vector(P.n_pad, P.C, 8)
    kc_v = np.where(P.C, P.apply(np.where(P.C, v, 0.0), a), 0.0)
    assert np.linalg.norm(P.jn(a, v) - kc_v) <= 1e-13 * np.linalg.norm(kc_v)
    assert np.linalg.norm(P.jnT(a, v) - kc_v) <= 1e-13 * np.linalg.norm(kc_v)


def test_dn_dk1_exact_linearity(oracle_mod):
    """N is affine in k1, so the central difference in k1 is exact up to rounding."""
    wl = iron8()
    P = oracle_mod.Problem(wl)
    a = saturated_state(P)
    k1 = wl.materials[0].k1
    Pp = oracle_mod.Problem(with_material(wl, k1=k1 + 0.5))
    Pm = oracle_mod.Problem(with_material(wl, k1=k1 - 0.5))
    fd = (Pp.n_c(a) - Pm.n_c(a)) / 1.0
    got = P.dn_dk1(a, 1)
    assert np.linalg.norm(got - fd) <= 1e-9 * np.linalg.norm(fd)


def test_dmsig_and_schur(oracle_mod):
    P = oracle_mod.Problem(iron8())
    sigma = P.wl.materials[0].sigma
    phi = P.dmsig(1)
    assert np.allclose(sigma * phi[P.C], P.msig[P.C], rtol=1e-14, atol=0)
    assert not phi[~P.C].any()
    w1 = synth.random_vector(P.n_pad, P.C, 41)
    w2 = synth.random_vector(P.n_pad, P.C, 42)
    s1, s2 = P.schur(w1), P.schur(w2)
    assert w2 @ s1 == pytest.approx(w1 @ s2, rel=1e-10)
    assert w1 @ s1 >= 0.0


def _loss(oracle_mod, wl, dt, M):
    from oracle.adjoint import forward_states, joule_loss
    P = oracle_mod.Problem(wl)
    return joule_loss(P, dt, forward_states(P, dt, M, rtol=1e-13))


def test_gradient_matches_central_difference(oracle_mod):
    """dL/dsigma and dL/dk1 of the adjoint vs central differences of the whole
    nonlinear run (the iron goes well past the knee of the Brauer curve)."""
    from oracle.adjoint import adjoint, forward_states
    wl = iron8()
    P = oracle_mod.Problem(wl)
    dt = 0.5 * 2 / P.power(iters=60)
    M = 16
    states = forward_states(P, dt, M, rtol=1e-13)
    B = P.cell_B(states[-1])[wl.cell_mat.astype(bool)]
    assert np.sqrt((B ** 2).sum(1)).max() > 1.0
    loss, g_sig, g_k1, _ = adjoint(P, dt, states, mat=1, rtol=1e-13)
    sigma, k1 = wl.materials[0].sigma, wl.materials[0].k1
    h = 1e-5
    fd_sig = (_loss(oracle_mod, with_material(wl, sigma=sigma * (1 + h)), dt, M)
              - _loss(oracle_mod, with_material(wl, sigma=sigma * (1 - h)), dt, M)) / (2 * h * sigma)
    fd_k1 = (_loss(oracle_mod, with_material(wl, k1=k1 * (1 + h)), dt, M)
             - _loss(oracle_mod, with_material(wl, k1=k1 * (1 - h)), dt, M)) / (2 * h * k1)
    assert g_sig == pytest.approx(fd_sig, rel=1e-6)
    assert g_k1 == pytest.approx(fd_k1, rel=1e-6)
    assert abs(g_k1) * k1 > 1e-6 * loss          # k1 has a visible effect


def test_gradient_closed_form_linear_mode(oracle_mod):
    """j = 0, a^0 = v (K_S v = lam_hat M_hat v, M_c = sigma M_hat):
    a^m = (1 - dt lam_hat / sigma)^m v, so
    L(sigma) = c dt lam_hat^2 / sigma * sum_{m<M} (1 - dt lam_hat/sigma)^(2m),
    c = v^T M_hat v, differentiated analytically."""
    from oracle.adjoint import adjoint, forward_states
    from oracle.dense import Dense
    wl = cube(6)
    wl.amp = 0.0
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    lam, V = D.gen_eig()
    sigma = wl.materials[0].sigma
    dt = 0.9 * 2 / lam.max()
    M = 9
    # skip the null modes of K_S (gradients inside the conductor): no decay, no loss
    first = int(np.argmax(lam > 1e-6 * lam.max()))
    for idx in (first, (first + len(lam)) // 2, len(lam) - 1):
        ac = np.zeros(P.n_pad)
        ac[D.c_slots] = V[:, idx] / np.abs(V[:, idx]).max()
        A0, _ = _state_from_ac(P, ac)
        states = forward_states(P, dt, M, rtol=1e-14, A0=A0)
        loss, g_sig, _, _ = adjoint(P, dt, states, rtol=1e-14)
        lh = lam[idx] * sigma                          # eigenvalue for M_hat
        c = (ac[D.c_slots] ** 2 * D.Mc / sigma).sum()
        x = dt * lh / sigma
        m = np.arange(M)
        S = ((1 - x) ** (2 * m)).sum()
        dS = (2 * m * (1 - x) ** (2 * m - 1) * (dt * lh / sigma ** 2)).sum()
        L = c * dt * lh ** 2 / sigma * S
        dL = c * dt * lh ** 2 * (-S / sigma ** 2 + dS / sigma)
        assert loss == pytest.approx(L, rel=1e-10)
        assert g_sig == pytest.approx(dL, rel=1e-8)
