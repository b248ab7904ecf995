"""Discrete adjoint on the GPU (C-ABI ec_adjoint_*) against the oracle's
adjoint (itself pinned by central differences and a closed form)."""
import numpy as np
import pytest

import synth
from tests.test_oracle_adjoint import iron8, with_material

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ec():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06721_amd as ec
    return ec


def oracle_grads(oracle_mod, wl, dt, M, rtol=1e-12):
    from oracle.adjoint import adjoint, forward_states
    P = oracle_mod.Problem(wl)
    states = forward_states(P, dt, M, rtol=rtol)
    loss, gs, gk, _ = adjoint(P, dt, states, mat=1, rtol=rtol)
    return loss, gs, gk, states


def gpu_grads(ec, G, dt, M, every, opts):
    ws = G.adjoint_workspace(M, every)
    A = G.zeros()
    loss = G.adjoint_forward(A, M, dt, every, opts, ws)
    g = G.adjoint_backward(M, dt, every, opts, ws, 1)
    return float(loss.item()), g.cpu().numpy(), A.cpu().numpy()


@pytest.mark.parametrize("method", [0, 2])
def test_adjoint_matches_oracle(ec, oracle_mod, method):
    """16 steps into Brauer saturation (|B| > 1 T): loss, dL/dsigma, dL/dk1."""
    wl = iron8()
    O = oracle_mod.Problem(wl)
    dt = 0.5 * 2 / O.power(iters=60)
    M = 16
    loss_o, gs_o, gk_o, states = oracle_grads(oracle_mod, wl, dt, M)
    G = ec.Problem(wl, window_cap=8)
    opts = ec.step_opts(method, window=8, rtol=1e-12)
    loss, g, A = gpu_grads(ec, G, dt, M, 5, opts)
    assert np.linalg.norm((A - states[-1])[O.C]) <= 1e-10 * np.linalg.norm(states[-1][O.C])
    assert loss == pytest.approx(loss_o, rel=1e-10)
    assert g[0] == pytest.approx(gs_o, rel=1e-8)
    assert g[1] == pytest.approx(gk_o, rel=1e-8)
    assert G.counters()["iters_adj"] > 0


def test_adjoint_checkpoint_interval_invariant(ec, oracle_mod):
    """Checkpoints hold the histories: every interval recomputes the same
    trajectory, so the gradients agree to rounding of nothing."""
    wl = iron8()
    O = oracle_mod.Problem(wl)
    dt = 0.5 * 2 / O.power(iters=60)
    M = 12
    opts = ec.step_opts(ec.SV_SPE, window=6, rtol=1e-10)
    out = []
    for every in (1, 5, M):
        G = ec.Problem(wl, window_cap=8)
        out.append(gpu_grads(ec, G, dt, M, every, opts))
    for loss, g, _ in out[1:]:
        assert loss == out[0][0]
        assert np.array_equal(g, out[0][1])


def test_adjoint_errors(ec, oracle_mod):
    G = ec.Problem(iron8(), window_cap=4)
    opts = ec.step_opts(ec.SV_ZERO, rtol=1e-10)
    ws = G.adjoint_workspace(4, 2)
    with pytest.raises(ec.ECError):           # backward before any forward
        G.adjoint_backward(4, 1e-6, 2, opts, ws, 1)
    A = G.zeros()
    G.adjoint_forward(A, 4, 1e-6, 2, opts, ws)
    with pytest.raises(ec.ECError):           # other step count than the forward
        G.adjoint_backward(3, 1e-6, 2, opts, ws, 1)
    with pytest.raises(ec.ECError):           # no such material
        G.adjoint_backward(4, 1e-6, 2, opts, ws, 2)


def test_set_material_matches_oracle(ec, oracle_mod):
    wl = iron8()
    O = oracle_mod.Problem(wl)
    dt = 0.5 * 2 / O.power(iters=60)
    m = wl.materials[0]
    wl2 = with_material(wl, sigma=3.1e6, k1=5.0)
    O2 = oracle_mod.Problem(wl2)
    Ao, *_ = O2.run(dt, 12, rtol=1e-12)
    G = ec.Problem(wl, window_cap=4)
    G.set_material(1, 3.1e6, 5.0, m.k2, m.k3)
    A = G.zeros()
    G.set_state(A, rtol=1e-12)
    G.run(A, 0, 12, dt, ec.step_opts(ec.SV_ZERO, rtol=1e-12))
    got = A.cpu().numpy()
    assert np.linalg.norm(got - Ao) <= 1e-10 * np.linalg.norm(Ao)


def test_eddy_loss_autograd(ec, oracle_mod):
    """torch.autograd through EddyLoss: gradients equal the oracle's adjoint."""
    import torch
    wl = iron8()
    O = oracle_mod.Problem(wl)
    dt = 0.5 * 2 / O.power(iters=60)
    M = 10
    loss_o, gs_o, gk_o, _ = oracle_grads(oracle_mod, wl, dt, M)
    G = ec.Problem(wl, window_cap=8)
    sigma = torch.tensor(wl.materials[0].sigma, dtype=torch.float64, requires_grad=True)
    k1 = torch.tensor(wl.materials[0].k1, dtype=torch.float64, requires_grad=True)
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=1e-12)
    loss = ec.eddy_loss(sigma, k1, G, dt, M, every=4, opts=opts)
    loss.backward()
    assert float(loss.detach()) == pytest.approx(loss_o, rel=1e-10)
    assert float(sigma.grad) == pytest.approx(gs_o, rel=1e-8)
    assert float(k1.grad) == pytest.approx(gk_o, rel=1e-8)
    # scaling of the upstream gradient passes through
    sigma.grad = None
    k1.grad = None
    (3.0 * ec.eddy_loss(sigma, k1, G, dt, M, every=4, opts=opts)).backward()
    assert float(sigma.grad) == pytest.approx(3.0 * gs_o, rel=1e-8)


def test_adjoint_full_size_central_difference(ec, oracle_mod):
    """64^3 grid (the adjoint workload's shape), 30 SPE steps at rtol 1e-12:
    the adjoint gradients against central differences of the GPU loss."""
    wl = synth.nonlinear(64, ramp_steps=30, J0=6.0e6)
    G = ec.Problem(wl, window_cap=8)
    dt = 0.5 * 2 / G.cfl(iters=40, rtol=1e-10)
    M, every = 30, 10
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=1e-12)
    loss, g, _ = gpu_grads(ec, G, dt, M, every, opts)
    m = wl.materials[0]
    ws = G.adjoint_workspace(M, every)

    def L(sigma, k1):
        G.set_material(1, sigma, k1, m.k2, m.k3)
        return float(G.adjoint_forward(G.zeros(), M, dt, every, opts, ws).item())
    # k1 moves the loss little in 30 steps: a step of 1e-4 keeps the
    # difference well above the noise of rtol-1e-12 solves (truncation ~h^2)
    h = 1e-4
    fd_s = (L(m.sigma * (1 + h), m.k1) - L(m.sigma * (1 - h), m.k1)) / (2 * h * m.sigma)
    fd_k = (L(m.sigma, m.k1 * (1 + h)) - L(m.sigma, m.k1 * (1 - h))) / (2 * h * m.k1)
    assert g[0] == pytest.approx(fd_s, rel=5e-5)
    assert g[1] == pytest.approx(fd_k, rel=5e-5)
