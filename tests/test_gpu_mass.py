"""The consistent conductivity matrix on the GPU (ec_set_mass, ec_mass_*):
its product, the Jacobi-PCG for M_c y = g with zero and SPE starts, and
explicit Euler steps that solve with M_c every step, against the oracle
(oracle/mass.py: the edge-element mass from its definition, scipy's sparse
direct solve, the Python stepper pinned against the C oracle)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from tests.conftest import small_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ec():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06721_amd as ec
    return ec


WORKLOADS = {
    "c1": lambda: synth.linear_c1(12),
    "small": lambda: small_workload(),
    "nl16": lambda: synth.nonlinear(16, ramp_steps=40, J0=6.0e6),
}


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def padded(P, v):
    x = np.zeros(P.n_pad)
    x[P.C] = v
    return x


@pytest.mark.parametrize("name", ["c1", "small", "nl16"])
def test_mass_apply(ec, oracle_mod, name):
    from oracle.mass import mass_matrix
    wl = WORKLOADS[name]()
    P = oracle_mod.Problem(wl)
    M = mass_matrix(P)
    G = ec.Problem(wl, window_cap=8)
    x = synth.random_vector(P.n_pad, P.C, 3)
    y = G.mass_apply(G.tensor(x)).cpu().numpy()
    ref = M @ x[P.C]
    assert rel(y[P.C], ref) <= 1e-14
    assert not y[~P.C].any()
    G.close()


@pytest.mark.parametrize("name", ["c1", "nl16"])
def test_mass_solve_zero_and_spe(ec, oracle_mod, name):
    """M_c y = g to rtol 1e-13 from zero and with SPE starts over a sequence
    of right-hand sides: every solution equals the direct solve; the SPE
    start's residual equals the oracle's projection of eq. (10) with M_c over
    the oracle's own previous solutions; SPE needs fewer iterations."""
    from oracle.mass import mass_matrix, spe_start_op
    wl = WORKLOADS[name]()
    P = oracle_mod.Problem(wl)
    M = mass_matrix(P)
    Mf = M.tocsc()
    G = ec.Problem(wl, window_cap=8)
    rng = np.random.default_rng(7)
    base = [rng.standard_normal(M.shape[0]) for _ in range(3)]
    gs = [M @ (base[0] + 0.1 * k * base[1] + 0.01 * k * k * base[2]) +
          1e-3 * rng.standard_normal(M.shape[0]) for k in range(8)]
    its = {}
    for method in (ec.SV_ZERO, ec.SV_SPE):
        G.set_mass(ec.MASS_CONSISTENT, method, window=5, rtol=1e-13, maxit=400)
        its[method] = []
        ys = []
        for k, g in enumerate(gs):
            info = G.info(1)
            y = G.mass_solve(G.tensor(padded(P, g)), info=info).cpu().numpy()[P.C]
            I = ec.info_array(info)[0]
            yo = spla.spsolve(Mf, g)
            assert I["status"] == 0 and I["rel_res"] <= 1e-13
            assert rel(y, yo) <= 1e-11, (method, k)
            if method == ec.SV_SPE and k > 0:
                x0 = spe_start_op(ys[-5:], g, lambda u: M @ u)
                r0 = np.linalg.norm(g - M @ x0) / np.linalg.norm(g)
                assert abs(I["r0_rel"] - r0) <= 1e-9 + 1e-6 * r0, k
            ys.append(yo)
            its[method].append(int(I["iters"]))
    print(f"PARITY mass solves {name}: iterations zero {its[0]} spe {its[2]}", flush=True)
    assert sum(its[ec.SV_SPE][2:]) < sum(its[ec.SV_ZERO][2:])
    G.close()


def consistent_dt(P, M, safety=0.5, iters=60):
    """safety * 2 / lambda_max of M^{-1} K_S(0) by the power method (oracle
    products and the direct solve)."""
    Mf = M.tocsc()
    v = np.random.default_rng(1).standard_normal(M.shape[0])
    lam = 0.0
    for _ in range(iters):
        v /= np.linalg.norm(v)
        x = padded(P, v)
        ks = P.apply(x, np.zeros(P.n_pad))[P.C] - P.schur(x)[P.C]
        y = spla.spsolve(Mf, ks)
        lam = float(v @ y)
        v = y
    return safety * 2.0 / lam


@pytest.mark.parametrize("name,method", [("c1", 2), ("nl16", 2), ("nl16", 0)])
def test_trajectory_consistent_mass(ec, oracle_mod, name, method):
    """30 explicit Euler steps with the consistent M_c (SPE-started M_c
    solves; K_n solves with `method`), rtol 1e-12 everywhere, against the
    oracle's stepper with the direct solve."""
    from oracle import mass
    wl = WORKLOADS[name]()
    P = oracle_mod.Problem(wl)
    M = mass.mass_matrix(P)
    dt = consistent_dt(P, M)
    Ao, _ = mass.run(P, M, dt, 30)
    G = ec.Problem(wl, window_cap=8)
    G.set_mass(ec.MASS_CONSISTENT, ec.SV_SPE, window=5, rtol=1e-12, maxit=400)
    A = G.zeros()
    G.set_state(A, rtol=1e-12)
    G.counters_reset()
    G.run(A, 0, 30, dt, ec.step_opts(method, window=8, rtol=1e-12))
    assert G.counters()["worst_status"] == 0
    mc = G.mass_counters()
    assert mc["solves"] == 30
    got = A.cpu().numpy()
    an, ano = np.where(P.N, got, 0.0), np.where(P.N, Ao, 0.0)
    e = {"a_c": rel(got[P.C], Ao[P.C]), "B": rel(P.curl(got), P.curl(Ao)),
         "Kn_an": rel(P.kn(an), P.kn(ano)), "A": rel(got, Ao)}
    print(f"PARITY consistent mass {name} method {method}: " +
          " ".join(f"{k}={v:.3e}" for k, v in e.items()) +
          f" mass iterations/step {mc['iters'] / 30:.2f}", flush=True)
    assert e["a_c"] <= 1e-10 and e["B"] <= 1e-10 and e["Kn_an"] <= 1e-10
    assert e["A"] <= (1e-10 if method == ec.SV_ZERO else 1e-6)
    # the lumped matrix again: the C oracle's loop
    G.set_mass(ec.MASS_LUMPED, ec.SV_SPE, window=5, rtol=1e-12, maxit=400)
    G.close()


def test_consistent_graph_equals_eager(ec, oracle_mod):
    wl = WORKLOADS["nl16"]()
    P = oracle_mod.Problem(wl)
    from oracle.mass import mass_matrix
    dt = consistent_dt(P, mass_matrix(P))
    runs = []
    for captured in (False, True):
        G = ec.Problem(wl, window_cap=8)
        G.set_mass(ec.MASS_CONSISTENT, ec.SV_SPE, window=5, rtol=1e-10, maxit=40)
        A = G.zeros()
        G.set_state(A, rtol=1e-10)
        opts = ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10)
        G.run(A, 0, 5, dt, opts)
        if captured:
            g = G.graph_capture(A, dt, ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10,
                                                    graph_iters=(4, 16)))
            for _ in range(10):
                g.launch()
            g.close()
        else:
            G.run(A, 5, 10, dt, opts)
        assert G.counters()["worst_status"] == 0
        runs.append(A.cpu().numpy())
        G.close()
    assert np.array_equal(runs[0], runs[1])
