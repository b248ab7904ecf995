"""The implicit Euler / Newton reference on the GPU (ec_implicit_step:
Newton on the Schur form, GMRES on J = M_c/dt + J_N - S with K_n^+ inside
every product) against the oracle (oracle/implicit.py, pinned by the dense
Schur solve, closed-form decay and quadratic convergence)."""
import time

import numpy as np
import pytest

import synth
from tests.test_oracle_pins import _state_from_ac, cube

pytestmark = pytest.mark.gpu

TIGHT = dict(newton_rtol=1e-12, gmres_rtol=1e-11, inner_rtol=1e-12, gmres_m=20, gmres_max=400)


@pytest.fixture(scope="module")
def ec():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06721_amd as ec
    return ec


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("method", [0, 2])
def test_implicit_linear_step(ec, oracle_mod, method):
    """Linear conductor, dt twenty times the explicit bound: one Newton step,
    the state of the oracle's implicit step (itself the dense Schur solve)."""
    from oracle import implicit
    from oracle.dense import Dense
    wl = cube(6)
    P = oracle_mod.Problem(wl)
    dt = 20 * 2 / Dense(P).gen_eig()[0].max()
    rng = np.random.default_rng(4)
    A0 = np.zeros(P.n_pad)
    A0[P.C] = rng.standard_normal(int(P.C.sum()))
    Ao, its, _ = implicit.step(P, A0, 3, dt, tol=1e-12)
    G = ec.Problem(wl, window_cap=8)
    A = G.tensor(A0)
    r = G.implicit_step(A, 3, dt, method=method, **TIGHT)
    assert r["status"] == 0 and r["newton_iters"] == its == 1
    got = A.cpu().numpy()
    assert rel(got[P.C], Ao[P.C]) <= 1e-10
    assert rel(P.curl(got), P.curl(Ao)) <= 1e-10
    G.close()


def test_implicit_eigenmode_decay(ec, oracle_mod):
    """j = 0, a^0 = v (K_S v = lambda M_c v), dt 50 times the explicit bound:
    a^m = (1 + dt lambda)^-m v."""
    from oracle.dense import Dense
    wl = cube(6)
    wl.amp = 0.0
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    lam, V = D.gen_eig()
    dt = 50 * 2 / lam.max()
    G = ec.Problem(wl, window_cap=8)
    for idx in (0, len(lam) - 1):
        ac = np.zeros(P.n_pad)
        ac[D.c_slots] = V[:, idx] / np.abs(V[:, idx]).max()
        A0, _ = _state_from_ac(P, ac)
        A = G.tensor(A0)
        G.set_state(A, rtol=1e-12)
        for m in range(1, 4):
            G.implicit_step(A, m, dt, **TIGHT)
            want = (1 + dt * lam[idx]) ** -m * ac[D.c_slots]
            got = A.cpu().numpy()[D.c_slots]
            assert np.linalg.norm(got - want) <= 1e-9 * np.linalg.norm(ac[D.c_slots]), (idx, m)
    G.close()


_NONLIN = {}


def _nonlinear_reference(oracle_mod):
    """The oracle's eight Newton steps (CPU, a few seconds), made once for
    both start methods."""
    if not _NONLIN:
        from oracle import implicit
        wl = synth.nonlinear(16, ramp_steps=8, J0=6.0e6)
        P = oracle_mod.Problem(wl)
        dt = 10 * 2 / P.power(iters=60)
        t0 = time.time()
        Ao, its = implicit.run(P, dt, 8, tol=1e-12)
        print(f"oracle implicit nl16: {time.time() - t0:.1f} s, newton {its}", flush=True)
        _NONLIN.update(wl=wl, P=P, dt=dt, Ao=Ao, its=its)
    return _NONLIN


@pytest.mark.parametrize("method", [0, 2])
def test_implicit_nonlinear_trajectory(ec, oracle_mod, method):
    """Brauer iron driven into saturation, dt ten times the explicit bound:
    eight implicit steps against the oracle's (Newton to 1e-12)."""
    ref = _nonlinear_reference(oracle_mod)
    wl, P, dt, Ao, its = ref["wl"], ref["P"], ref["dt"], ref["Ao"], ref["its"]
    B = P.cell_B(Ao)[wl.cell_mat.astype(bool)]
    G = ec.Problem(wl, window_cap=8)
    A = G.zeros()
    G.set_state(A, rtol=1e-12)
    nits = []
    # SPE-started coupling solves: the start vector's error lies outside the
    # window, so ||F|| levels off near the inner tolerance times the
    # conditioning (about 1e-12 relative here); Newton stops at 1e-10
    kw = dict(TIGHT, newton_rtol=1e-10) if method == ec.SV_SPE else TIGHT
    for m in range(1, 9):
        t0 = time.time()
        r = G.implicit_step(A, m, dt, method=method, **kw)
        print(f"implicit step {m} (method {method}): {time.time() - t0:.2f} s, {r}", flush=True)
        assert r["status"] == 0, r
        nits.append(r["newton_iters"])
    got = A.cpu().numpy()
    an, ano = np.where(P.N, got, 0.0), np.where(P.N, Ao, 0.0)
    e = {"a_c": rel(got[P.C], Ao[P.C]), "B": rel(P.curl(got), P.curl(Ao)),
         "Kn_an": rel(P.kn(an), P.kn(ano)), "A": rel(got, Ao)}
    print(f"PARITY implicit nl16 method {method}: " +
          " ".join(f"{k}={v:.3e}" for k, v in e.items()) +
          f" newton {nits} oracle {its} |B|max {np.sqrt((B ** 2).sum(1)).max():.2f}", flush=True)
    assert e["a_c"] <= 1e-9 and e["B"] <= 1e-9 and e["Kn_an"] <= 1e-9
    assert e["A"] <= (1e-9 if method == 0 else 1e-6)
    assert all(abs(a - b) <= 1 for a, b in zip(nits, its))
    if method == ec.SV_ZERO:
        assert nits == its
    G.close()
