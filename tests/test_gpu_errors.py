"""Error semantics of the C-ABI on the GPU: the explicit Euler bound of
eq. (8) (growth beyond it, EC_ERR_CFL from the last ec_cfl), non-finite
states (EC_ERR_NONFINITE in the solve records) and a singular projected SPE
matrix (EC_ERR_SINGULAR_PROJ recorded, zero start used, the solve goes on).
Expected values come from the oracle's dense matrices and CG."""
import numpy as np
import pytest

import synth
from tests.test_oracle_pins import _state_from_ac, cube

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ec():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06721_amd as ec
    return ec


def top_mode(oracle_mod):
    from oracle.dense import Dense
    wl = cube(6)
    wl.amp = 0.0                   # j = 0: the step is a_c <- (I - dt M_c^-1 K_S) a_c
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    lam, V = D.gen_eig()
    ac = np.zeros(P.n_pad)
    ac[D.c_slots] = V[:, -1] / np.abs(V[:, -1]).max()
    return wl, P, D, lam.max(), ac


@pytest.mark.parametrize("factor,grows", [(0.99, False), (1.01, True)])
def test_cfl_bound_sharp_on_gpu(ec, oracle_mod, factor, grows):
    """a_c^0 = the top generalized eigenvector of (K_S, M_c): at dt = 1.01 x
    2/lambda_max it grows by |1 - dt lambda_max| per step, at 0.99 x it
    decays, each step within 1e-8 of the closed form (1 - dt lambda)^m v."""
    wl, P, D, lmax, ac = top_mode(oracle_mod)
    A0, _ = _state_from_ac(P, ac)
    G = ec.Problem(wl, window_cap=5)
    A = G.tensor(A0)
    G.set_state(A, rtol=1e-13)
    dt = factor * 2.0 / lmax
    g = 1.0 - dt * lmax
    v = ac[D.c_slots]
    for m in range(1, 21):
        G.step(A, m, dt, ec.step_opts(ec.SV_SPE, window=5, rtol=1e-13))
        got = A.cpu().numpy()[D.c_slots]
        want = g ** m * v
        assert np.linalg.norm(got - want) <= 1e-8 * np.linalg.norm(want), m
    ratio = np.linalg.norm(got) / np.linalg.norm(v)
    assert (ratio > 1.0) == grows
    assert ratio == pytest.approx(abs(g) ** 20, rel=1e-7)
    G.close()


def test_cfl_error_code(ec, oracle_mod):
    """After ec_cfl, a step with dt above 2/lambda_max returns EC_ERR_CFL and
    leaves the state untouched; below the bound it runs; ec_set_material
    drops the stored bound."""
    wl, P, D, lmax, ac = top_mode(oracle_mod)
    G = ec.Problem(wl, window_cap=5)
    A0, _ = _state_from_ac(P, ac)
    lam = G.cfl(A=G.tensor(A0), iters=300, rtol=1e-12)
    assert lam == pytest.approx(lmax, rel=1e-5)
    A = G.tensor(A0)
    G.set_state(A, rtol=1e-12)
    opts = ec.step_opts(ec.SV_ZERO, rtol=1e-12)
    with pytest.raises(ec.ECError) as ei:
        G.step(A, 1, 1.01 * 2.0 / lam, opts)
    assert ei.value.code == ec.EC_ERR_CFL
    with pytest.raises(ec.ECError) as ei:
        G.graph_capture(A, 1.01 * 2.0 / lam, opts)
    assert ei.value.code == ec.EC_ERR_CFL
    assert np.array_equal(A.cpu().numpy(), A0)
    G.step(A, 1, 0.99 * 2.0 / lam, opts)
    assert G.counters()["worst_status"] == 0
    m = wl.materials[0]
    G.set_material(1, m.sigma, m.k1, m.k2, m.k3)
    G.step(A, 2, 1.01 * 2.0 / lam, opts)           # no bound stored any more
    G.close()


@pytest.mark.parametrize("method", [0, 2])
def test_nonfinite_state_reported(ec, oracle_mod, method):
    """A NaN on one conducting edge of the state reaches the coupling solve's
    right-hand side (K_cn^T a_c): its record and the worst-status counter
    report EC_ERR_NONFINITE; the call itself returns (asynchronous)."""
    wl = synth.linear_c1(12)
    O = oracle_mod.Problem(wl)
    G = ec.Problem(wl, window_cap=5)
    A0 = np.zeros(O.n_pad)
    A0[np.flatnonzero(O.C)[7]] = np.nan
    A = G.tensor(A0)
    G.set_state(A, rtol=1e-10)
    G.counters_reset()
    info = G.info(2)
    G.step(A, 1, 1e-9, ec.step_opts(method, window=5, rtol=1e-10), info=info)
    I = ec.info_array(info)
    assert I["status"][0] == ec.EC_OK                  # the source solve is unaffected
    assert I["status"][1] == ec.EC_ERR_NONFINITE
    assert G.counters()["worst_status"] == ec.EC_ERR_NONFINITE
    G.close()


def test_singular_projection_zero_start(ec, oracle_mod):
    """With the projection as printed (grad-div factor 0), a window holding a
    pure gradient (a null vector of K_n) makes U^T K_n U singular: the solve
    records EC_ERR_SINGULAR_PROJ, starts from zero (r0 = b) and still returns
    the oracle's minimum-norm solution."""
    from oracle.dense import gradient
    from oracle.startvec import free_nodes
    wl = synth.linear_c1(12)
    O = oracle_mod.Problem(wl)
    G = ec.Problem(wl, window_cap=5)
    G.set_gauge_penalty(0.0)
    nx, ny, nz = wl.n
    S = (nx + 1) * (ny + 1) * (nz + 1)
    phi = np.where(free_nodes(O), np.random.default_rng(5).standard_normal(S), 0.0)
    g = gradient(wl.n, phi)
    assert np.abs(O.kn(g)).max() <= 1e-9 * np.abs(O.kn(np.abs(g))).max()
    seq = ec.SEQ_USER
    G.history_reset(seq)
    G.history_push(seq, ec.SV_SPE, 5, G.tensor(g))
    b = O.kcnT(synth.random_vector(O.n_pad, O.C, 11))
    info = G.info(1)
    x = G.solve(G.tensor(b), seq=seq, method=ec.SV_SPE, window=5, rtol=1e-12,
                info=info).cpu().numpy()
    I = ec.info_array(info)[0]
    assert I["status"] == ec.EC_ERR_SINGULAR_PROJ
    assert I["r0_rel"] == pytest.approx(1.0, rel=1e-12)
    assert I["rel_res"] <= 1e-12
    xo, *_ = O.cg(b, rtol=1e-12)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
    G.close()
