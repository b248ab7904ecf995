"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Inputs are seeded (synth); expected values come from the oracle only.
Tolerances: FP64 operator products agree to rounding (1e-13 relative to the
largest entry); solves and trajectories at rtol 1e-12 agree to 1e-10 relative
(the bound stated for the FP64 path); start vectors to 1e-10.
"""
import numpy as np
import pytest

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


def lshape_workload():
    """Non-box conductor (two overlapping boxes): exercises the class table."""
    wl = small_workload(n=(9, 8, 7), length=(1.0, 0.9, 0.7), lo=(3, 3, 2), hi=(5, 4, 3))
    cm = wl.cell_mat.reshape(7, 8, 9)
    cm[4, 3:5, 3:6] = 1          # extend the box upwards
    cm[2:5, 5, 3] = 1
    wl.cell_mat = cm.reshape(-1).copy()
    return wl


def nonlinear16():
    """Iron driven to ~2 T within 60 steps, still stable at half the bound."""
    return synth.nonlinear(16, ramp_steps=40, J0=6.0e6)


WORKLOADS = {
    "c1": lambda: synth.linear_c1(12),
    "small": lambda: small_workload(),
    "lshape": lshape_workload,
    "nl16": nonlinear16,
}


def pair(ec, oracle_mod, name, cap=8):
    wl = WORKLOADS[name]()
    return ec.Problem(wl, window_cap=cap), oracle_mod.Problem(wl), wl


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ------------------------------------------------------------ operators
@pytest.mark.parametrize("name", ["c1", "small", "lshape", "nl16"])
def test_kn_and_kcnT(ec, oracle_mod, name):
    G, O, _ = pair(ec, oracle_mod, name)
    for seed in (1, 2):
        x = synth.random_vector(O.n_pad, O.N, seed)
        y = G.apply(ec.OP_KN, G.tensor(x)).cpu().numpy()
        assert rel(y, O.kn(x)) < 1e-13
        a = synth.random_vector(O.n_pad, O.C, seed + 10)
        y = G.apply(ec.OP_KCN_T, G.tensor(a)).cpu().numpy()
        assert rel(y, O.kcnT(a)) < 1e-13
        # a full random vector: the operators read only their own block
        z = synth.random_vector(O.n_pad, ~O.D, seed + 20)
        y = G.apply(ec.OP_KN, G.tensor(z)).cpu().numpy()
        assert rel(y, O.kn(np.where(O.N, z, 0.0))) < 1e-13


@pytest.mark.parametrize("name", ["c1", "lshape", "nl16"])
def test_kc_kcn_nonlinear(ec, oracle_mod, name):
    """[K_nu(a) a]_C with the Brauer reluctivity evaluated at a (|B| ~ 1 T)."""
    G, O, wl = pair(ec, oracle_mod, name)
    rng = np.random.default_rng(5)
    a = synth.random_vector(O.n_pad, ~O.D, 7)
    h = min(wl.h)
    a *= 0.4 * h * h / np.abs(a).max()       # |B| of order 1 T
    y = G.apply(ec.OP_KC_KCN, G.tensor(a)).cpu().numpy()
    ref = np.where(O.C, O.apply(a, a), 0.0)
    assert rel(y, ref) < 1e-12


def test_full_size_spmv(ec, oracle_mod):
    """K_n at the 48^3 and 128^3 sizes, full comparison."""
    for N in (48, 128):
        wl = synth.nonlinear(N)
        G = ec.Problem(wl, window_cap=1)
        O = oracle_mod.Problem(wl)
        x = synth.random_vector(O.n_pad, O.N, N)
        y = G.apply(ec.OP_KN, G.tensor(x)).cpu().numpy()
        assert rel(y, O.kn(x)) < 1e-13
        del G


# --------------------------------------------------------------- solves
@pytest.mark.parametrize("name", ["c1", "small", "lshape"])
def test_solve_zero_start(ec, oracle_mod, name):
    G, O, _ = pair(ec, oracle_mod, name)
    b = O.kcnT(synth.random_vector(O.n_pad, O.C, 3)) + O.source(2, 1e-3)
    info = G.info(1)
    x = G.solve(G.tensor(b), method=ec.SV_ZERO, rtol=1e-12, info=info).cpu().numpy()
    I = ec.info_array(info)[0]
    xo, ito, relo, st = O.cg(b, rtol=1e-12)
    assert I["status"] == 0 and I["rel_res"] <= 1e-12
    # true residual through the oracle operator
    assert np.linalg.norm(b - O.kn(x)) <= 2e-12 * np.linalg.norm(b)
    if name == "c1":
        # cubic cells: the Jacobi diagonal is one scalar, PCG from zero stays in
        # range(K_n) and returns the same minimum-norm solution as plain CG
        assert abs(int(I["iters"]) - ito) <= max(2, ito // 20)
        assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
    else:
        # non-cubic cells: Jacobi differs per edge direction, so PCG picks
        # another pseudo-inverse solution (a gradient field apart): compare the
        # gauge-invariant flux C x and K_n x
        assert np.linalg.norm(O.curl(x) - O.curl(xo)) <= 1e-10 * np.linalg.norm(O.curl(xo))
        assert np.linalg.norm(O.kn(x) - O.kn(xo)) <= 1e-11 * np.linalg.norm(b)


def test_solve_prev_start_and_zero_rhs(ec, oracle_mod):
    G, O, _ = pair(ec, oracle_mod, "c1")
    b = O.source(3, 1e-3)
    xo, *_ = O.cg(b, rtol=1e-13)
    x0 = 0.9 * xo
    info = G.info(1)
    x = G.solve(G.tensor(b), x=G.tensor(x0), method=ec.SV_PREV, rtol=1e-12, info=info)
    I = ec.info_array(info)[0]
    assert I["status"] == 0
    assert I["r0_rel"] == pytest.approx(np.linalg.norm(b - O.kn(x0)) / np.linalg.norm(b), rel=1e-8)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    # b = 0: x = 0 after 0 iterations, for any start
    z = G.zeros()
    x = G.solve(z, x=G.tensor(x0), method=ec.SV_PREV, rtol=1e-12, info=info)
    I = ec.info_array(info)[0]
    assert I["iters"] == 0 and I["status"] == 0 and not x.cpu().numpy().any()
    x = G.solve(z, method=ec.SV_ZERO, info=info)
    assert ec.info_array(info)[0]["iters"] == 0 and not x.cpu().numpy().any()


def test_solve_maxit_reports_not_converged(ec, oracle_mod):
    G, O, _ = pair(ec, oracle_mod, "c1")
    b = O.source(3, 1e-3)
    info = G.info(1)
    G.solve(G.tensor(b), method=ec.SV_ZERO, rtol=1e-14, maxit=3, info=info)
    I = ec.info_array(info)[0]
    assert I["status"] == -3 and I["iters"] == 3
    # and the same three iterations as the oracle's CG
    xo, it, _, st = O.cg(b, rtol=1e-14, maxit=3)
    assert st == -3


# ------------------------------------------------------- start vectors
def time_window(O, dt, steps):
    """Consecutive CPL solutions of the oracle's own time loop."""
    A = np.zeros(O.n_pad)
    sc = np.zeros(O.n_pad)
    out = []
    for m in range(steps):
        A, sc, *_ = O.run(dt, 1, rtol=1e-13, A=A, sc=sc, m0=m)
        out.append(sc.copy())
    return out, A


def test_spe_start_parity_and_sliding_window(ec, oracle_mod):
    from oracle.startvec import spe_start
    G, O, _ = pair(ec, oracle_mod, "c1")
    dt = 0.9 * 2 / O.power(iters=40)
    sols, A = time_window(O, dt, 9)
    b = O.kcnT(synth.random_vector(O.n_pad, O.C, 9))
    seq = ec.SEQ_USER
    G.history_reset(seq)
    for k, v in enumerate(sols):
        G.history_push(seq, ec.SV_SPE, 5, G.tensor(v))
        if k in (0, 2, 4, 8):
            x0 = G.start_vector(seq, ec.SV_SPE, 5, G.tensor(b)).cpu().numpy()
            ref = spe_start(O, sols[max(0, k - 4):k + 1], b)
            assert np.linalg.norm(x0 - ref) <= 1e-9 * np.linalg.norm(ref), k
    # Galerkin orthogonality of the GPU start vector on the window
    r = b - O.kn(x0)
    for v in sols[-5:]:
        assert abs(v @ r) <= 1e-9 * np.linalg.norm(v) * np.linalg.norm(b)


def test_spe_exact_and_random_window(ec, oracle_mod):
    from oracle.startvec import spe_start
    G, O, _ = pair(ec, oracle_mod, "small")
    win = [O.kn(synth.random_vector(O.n_pad, O.N, 30 + s)) for s in range(6)]
    seq = ec.SEQ_ADJ
    G.history_reset(seq)
    for v in win:
        G.history_push(seq, ec.SV_SPE, 6, G.tensor(v))
    x = win[1] - 0.5 * win[4]
    x0 = G.start_vector(seq, ec.SV_SPE, 6, G.tensor(O.kn(x))).cpu().numpy()
    assert np.linalg.norm(x0 - x) <= 1e-10 * np.linalg.norm(x)
    b = O.source(1, 1e-3) + O.kcnT(synth.random_vector(O.n_pad, O.C, 4))
    x0 = G.start_vector(seq, ec.SV_SPE, 6, G.tensor(b)).cpu().numpy()
    ref = spe_start(O, win, b)
    assert np.linalg.norm(x0 - ref) <= 1e-10 * np.linalg.norm(ref)
    # a dependent push does not grow the basis
    G.history_push(seq, ec.SV_SPE, 6, G.tensor(2.0 * win[5] - win[0]))
    x1 = G.start_vector(seq, ec.SV_SPE, 6, G.tensor(b)).cpu().numpy()
    assert np.linalg.norm(x1 - ref) <= 1e-9 * np.linalg.norm(ref)


def test_spe_large_window(ec, oracle_mod):
    """Windows wider than the register Cholesky (12 columns): the start
    factors H in shared memory; the sliding window (13 of 15 pushes) and the
    stored-factor start of a 12-column window agree with the oracle."""
    from oracle.startvec import spe_start
    G, O, _ = pair(ec, oracle_mod, "small", cap=16)
    win = [O.kn(synth.random_vector(O.n_pad, O.N, 60 + s)) for s in range(15)]
    b = O.source(1, 1e-3) + O.kcnT(synth.random_vector(O.n_pad, O.C, 7))
    for w in (13, 12):
        seq = ec.SEQ_ADJ
        G.history_reset(seq)
        for v in win:
            G.history_push(seq, ec.SV_SPE, w, G.tensor(v))
        x0 = G.start_vector(seq, ec.SV_SPE, w, G.tensor(b)).cpu().numpy()
        ref = spe_start(O, win[-w:], b)
        assert np.linalg.norm(x0 - ref) <= 1e-9 * np.linalg.norm(ref), w


def test_cspe_growing_basis(ec, oracle_mod):
    """The paper's growing basis (fewer than 20 columns, only the newest
    column added per step): with a 19-column window each push appends one
    orthogonalised column, the start vector is the projection on all
    solutions so far, and the 20th push slides the window.  The start vectors
    agree with the oracle's projection after 1, 6, 12, 13, 19 and 20 pushes
    (both Cholesky paths: up to 12 columns in registers, beyond in shared
    memory)."""
    from oracle.startvec import spe_start
    G, O, _ = pair(ec, oracle_mod, "small", cap=20)
    win = [O.kn(synth.random_vector(O.n_pad, O.N, 80 + s)) for s in range(20)]
    b = O.source(1, 1e-3) + O.kcnT(synth.random_vector(O.n_pad, O.C, 9))
    seq = ec.SEQ_USER
    G.history_reset(seq)
    for i, v in enumerate(win, 1):
        G.history_push(seq, ec.SV_SPE, 19, G.tensor(v))
        if i in (1, 6, 12, 13, 19, 20):
            x0 = G.start_vector(seq, ec.SV_SPE, 19, G.tensor(b)).cpu().numpy()
            ref = spe_start(O, win[max(0, i - 19):i], b)
            assert np.linalg.norm(x0 - ref) <= 1e-9 * np.linalg.norm(ref), i


def test_spe_gauge_penalty(ec, oracle_mod):
    """A window holding a pure gradient (a null vector of K_n): with the
    grad-div term the start vector is x* itself, as in the oracle; with the
    term switched off a normal window still matches the printed projection."""
    from oracle.dense import gradient
    from oracle.startvec import free_nodes, spe_start
    G, O, wl = pair(ec, oracle_mod, "c1")
    dt = 0.9 * 2 / O.power(iters=40)
    sols, _ = time_window(O, dt, 6)
    nx, ny, nz = wl.n
    S = (nx + 1) * (ny + 1) * (nz + 1)
    phi = np.where(free_nodes(O), np.random.default_rng(3).standard_normal(S), 0.0)
    g = gradient(wl.n, phi)
    xs = sols[-1]
    seq = ec.SEQ_USER
    G.history_reset(seq)
    for v in (sols[-3], g, xs):
        G.history_push(seq, ec.SV_SPE, 5, G.tensor(v))
    b = O.kn(xs)
    x0 = G.start_vector(seq, ec.SV_SPE, 5, G.tensor(b)).cpu().numpy()
    assert np.linalg.norm(x0 - xs) <= 1e-9 * np.linalg.norm(xs)
    b2 = O.kcnT(synth.random_vector(O.n_pad, O.C, 14))
    x1 = G.start_vector(seq, ec.SV_SPE, 5, G.tensor(b2)).cpu().numpy()
    ref = spe_start(O, [sols[-3], g, xs], b2)
    assert np.linalg.norm(x1 - ref) <= 1e-9 * np.linalg.norm(ref)
    G.set_gauge_penalty(0.0)
    for v in sols[-5:]:
        G.history_push(seq, ec.SV_SPE, 5, G.tensor(v))
    x2 = G.start_vector(seq, ec.SV_SPE, 5, G.tensor(b2)).cpu().numpy()
    ref0 = spe_start(O, sols[-5:], b2, penalty=0.0)
    assert np.linalg.norm(x2 - ref0) <= 1e-9 * np.linalg.norm(ref0)
    with pytest.raises(ec.ECError):
        G.set_gauge_penalty(-1.0)


@pytest.mark.parametrize("eps,kmax,window", [(0.0, 6, "random"), (1e-4, 3, "time"),
                                             (1e-4, 6, "time")])
def test_pod_start_parity(ec, oracle_mod, eps, kmax, window):
    """Gram-eigen POD (GPU) vs SVD POD (oracle).  Without truncation the test
    uses a well-conditioned window: the method of snapshots squares the
    condition number, so modes below ~1e-8 sigma_1 are not resolved; the
    paper's eps_POD = 1e-4 keeps only resolved modes."""
    from oracle.startvec import pod_start
    G, O, _ = pair(ec, oracle_mod, "c1")
    if window == "time":
        dt = 0.9 * 2 / O.power(iters=40)
        sols, _ = time_window(O, dt, 8)
    else:
        sols = [O.kn(synth.random_vector(O.n_pad, O.N, 50 + s)) for s in range(8)]
    win = sols[-6:]
    seq = ec.SEQ_USER
    G.history_reset(seq)
    for v in sols:
        G.history_push(seq, ec.SV_POD, 6, G.tensor(v))
    b = O.kcnT(synth.random_vector(O.n_pad, O.C, 12))
    info = G.info(1)
    x0 = G.start_vector(seq, ec.SV_POD, 6, G.tensor(b), pod_kmax=kmax, pod_eps=eps,
                        info=info).cpu().numpy()
    ref, k, inf = pod_start(O, win, b, eps=eps, kmax=kmax)
    I = ec.info_array(info)[0]
    assert I["basis_cols"] == k
    assert I["pod_info"] == pytest.approx(inf, rel=1e-8)
    assert np.linalg.norm(x0 - ref) <= 1e-8 * np.linalg.norm(ref)


# ----------------------------------------------------------- trajectories
@pytest.mark.parametrize("method,window", [(0, 5), (1, 5), (2, 5), (3, 5)])
def test_trajectory_c1(ec, oracle_mod, method, window):
    """200 explicit Euler steps of the linear case, every start vector, at
    rtol 1e-12 on both sides: relative error of A <= 1e-10 (sampled every 40)."""
    G, O, _ = pair(ec, oracle_mod, "c1")
    dt = 0.9 * 2 / O.power(iters=60)
    opts = ec.step_opts(method, window=window, pod_kmax=window, pod_eps=1e-4, rtol=1e-12)
    A = G.zeros()
    Ao = np.zeros(O.n_pad)
    sc = np.zeros(O.n_pad)
    for blk in range(5):
        G.run(A, 40 * blk, 40, dt, opts)
        Ao, sc, *_ = O.run(dt, 40, rtol=1e-12, A=Ao, sc=sc, m0=40 * blk)
        got = A.cpu().numpy()
        assert np.linalg.norm(got - Ao) <= 1e-10 * np.linalg.norm(Ao), blk
        assert np.linalg.norm(O.curl(got) - O.curl(Ao)) <= 1e-10 * np.linalg.norm(O.curl(Ao))
    assert G.counters()["worst_status"] == 0


def test_trajectory_nonlinear16(ec, oracle_mod):
    """Saturating Brauer iron (peak |B| > 1 T) at N = 16.

    Zero-start PCG with a scalar Jacobi diagonal returns the minimum-norm
    pseudo-inverse solution, so that trajectory must match the oracle's edge
    by edge.  SPE start vectors carry a gradient (null-space) part into a_n
    that PCG never removes; everything that part cannot reach (a_c, the face
    fluxes b = C a, and K_n a_n) must still match."""
    G, O, wl = pair(ec, oracle_mod, "nl16")
    dt = 0.5 * 2 / O.power(iters=60)
    Ao, *_ = O.run(dt, 60, rtol=1e-12)
    B = O.cell_B(Ao)[wl.cell_mat.astype(bool)]
    assert np.sqrt((B ** 2).sum(1)).max() > 1.0
    nrm = np.linalg.norm
    for method in (ec.SV_ZERO, ec.SV_SPE):
        A = G.zeros()
        G.set_state(A, rtol=1e-12)           # s_c = 0 and empty histories again
        G.counters_reset()
        G.run(A, 0, 60, dt, ec.step_opts(method, window=8, rtol=1e-12))
        got = A.cpu().numpy()
        assert G.counters()["worst_status"] == 0
        if method == ec.SV_ZERO:
            assert nrm(got - Ao) <= 1e-10 * nrm(Ao)
            continue
        c = O.C
        assert nrm((got - Ao)[c]) <= 1e-10 * nrm(Ao[c])
        assert nrm(O.curl(got) - O.curl(Ao)) <= 1e-10 * nrm(O.curl(Ao))
        an, ano = np.where(O.N, got, 0.0), np.where(O.N, Ao, 0.0)
        assert nrm(O.kn(an) - O.kn(ano)) <= 1e-9 * nrm(O.kn(ano))
        # the grad-div term of the projection keeps the gradient part at the
        # level of the solver tolerance (it grows without bound otherwise)
        assert nrm(got - Ao) <= 1e-6 * nrm(Ao)


@pytest.mark.parametrize("name,method", [("c1", 2), ("nl16", 2), ("nl16", 3)])
def test_graph_replay_equals_eager(ec, oracle_mod, name, method):
    """Captured steps replayed after eager warm-up steps: with iteration
    budgets that cover every solve the trajectory is bitwise the eager one;
    with budgets far too small the persistent tail finishes the solves, and
    on these grids (at most one 256-node tile per block) it runs the same
    iteration body as the captured kernels, so the trajectory is still
    bitwise the eager one; history pushes that a captured step runs beside
    the other sequence's work (and the one it leaves due) keep the eager
    order, so eager steps after the replays continue the eager trajectory
    bitwise; maxit still reports NOT_CONVERGED."""
    G1, O, wl = pair(ec, oracle_mod, name)
    dt = 0.5 * 2 / O.power(iters=40)
    opts = ec.step_opts(method, window=8, pod_kmax=6, rtol=1e-10)
    A1 = G1.zeros()
    G1.set_state(A1, rtol=1e-10)
    info1 = G1.info(60)
    G1.run(A1, 0, 30, dt, opts, info=info1)
    its = ec.info_array(info1)["iters"]
    ref = A1.cpu().numpy()
    G1.run(A1, 30, 5, dt, opts)
    ref35 = A1.cpu().numpy()
    cover = (int(its[20::2].max()) + 2, int(its[21::2].max()) + 2)
    for budget, serial in ((cover, False), ((1, 2), False), (cover, True)):
        G2 = ec.Problem(wl, window_cap=8)
        A2 = G2.zeros()
        G2.set_state(A2, rtol=1e-10)
        G2.run(A2, 0, 10, dt, opts)
        G2.counters_reset()
        g = G2.graph_capture(A2, dt, ec.step_opts(method, window=8, pod_kmax=6, rtol=1e-10,
                                                  graph_iters=budget, graph_serial=serial))
        for _ in range(20):
            g.launch()
        got = A2.cpu().numpy()
        c = G2.counters()
        assert c["worst_status"] == 0 and c["steps"] == 20
        n_ref = int(its[20:].sum())
        assert np.array_equal(got, ref), budget
        assert c["iters_src"] + c["iters_cpl"] == n_ref
        # a forked (SPE) replay leaves its coupling solution due for a push (made beside
        # the next step's source solve); eager steps after replays make it
        # first, so the run continues as the eager one
        G2.run(A2, 30, 5, dt, opts)
        assert np.array_equal(A2.cpu().numpy(), ref35), budget
        del g
    # maxit below the need: reported, not hidden (also through the tail)
    A3 = G2.zeros()
    G2.set_state(A3, rtol=1e-10)
    G2.set_step(0)
    G2.counters_reset()
    g = G2.graph_capture(A3, dt, ec.step_opts(method, window=8, pod_kmax=6, rtol=1e-10,
                                               maxit=5, graph_iters=(1, 1)))
    g.launch()
    c = G2.counters()
    assert c["worst_status"] == ec.EC_ERR_NOT_CONVERGED
    assert c["iters_cpl"] == 5


def test_graph_forked_starved_48(ec):
    """The benchmark's 48^3 Brauer grid and step shape (SPE m = 8, rtol 1e-8),
    captured with the history pushes on the forked side stream and budgets far
    too small (one source and two coupling iteration kernels): the persistent
    tail runs beside the pushes of the other sequence, which hold CUs while
    its blocks arrive at the grid barrier; the replays must still be bitwise
    the eager steps, with no error record."""
    import torch
    wl = synth.nonlinear(48)
    opts = ec.step_opts(ec.SV_SPE, window=8, pod_kmax=8, rtol=1e-8)
    G1 = ec.Problem(wl, window_cap=8)
    dt = 0.5 * 2.0 / G1.cfl(iters=60, rtol=1e-10)
    A1 = G1.zeros()
    G1.set_state(A1, rtol=1e-8)
    info1 = G1.info(2 * 20)
    G1.run(A1, 0, 20, dt, opts, info=info1)
    its = ec.info_array(info1)["iters"]
    ref = A1.cpu().numpy()
    G1.close()
    G2 = ec.Problem(wl, window_cap=8)
    A2 = G2.zeros()
    G2.set_state(A2, rtol=1e-8)
    G2.run(A2, 0, 5, dt, opts)
    G2.counters_reset()
    g = G2.graph_capture(A2, dt, ec.step_opts(ec.SV_SPE, window=8, pod_kmax=8, rtol=1e-8,
                                              graph_iters=(1, 2), graph_serial=False))
    for _ in range(15):
        g.launch()
    torch.cuda.synchronize()
    c = G2.counters()
    assert c["worst_status"] == 0 and c["steps"] == 15
    assert c["iters_src"] + c["iters_cpl"] == int(its[10:].sum())
    assert int(its[11::2].max()) > 2        # the tail carried coupling iterations
    assert np.array_equal(A2.cpu().numpy(), ref)
    g.close()
    G2.close()


def test_step_info_records(ec, oracle_mod):
    G, O, _ = pair(ec, oracle_mod, "c1")
    dt = 0.9 * 2 / O.power(iters=40)
    info = G.info(2 * 10)
    A = G.zeros()
    G.run(A, 0, 10, dt, ec.step_opts(ec.SV_SPE, window=5, rtol=1e-10), info=info)
    I = ec.info_array(info)
    assert (I["status"] == 0).all()
    assert (I["rel_res"] <= 1e-10).all()
    src, cpl = I[0::2], I[1::2]
    assert (src["iters"][2:] == 0).all()         # j^m is parallel to the stored solution
    assert (src["basis_cols"][1:] == 1).all()
    c = G.counters()
    assert c["steps"] == 10 and c["iters_src"] == src["iters"].sum()
    assert c["iters_cpl"] == cpl["iters"].sum()


def test_set_state_and_continue(ec, oracle_mod):
    """ec_set_state from an oracle state, then steps: same as continuing the oracle."""
    G, O, _ = pair(ec, oracle_mod, "c1")
    dt = 0.9 * 2 / O.power(iters=40)
    Ao, sc, *_ = O.run(dt, 15, rtol=1e-13)
    A = G.tensor(Ao)
    G.set_state(A, rtol=1e-13)
    G.run(A, 15, 10, dt, ec.step_opts(ec.SV_PREV, rtol=1e-12))
    A2, *_ = O.run(dt, 10, rtol=1e-12, A=Ao, sc=sc, m0=15)
    assert np.linalg.norm(A.cpu().numpy() - A2) <= 1e-10 * np.linalg.norm(A2)


def test_cfl_power_method(ec, oracle_mod):
    """Eq. (8) bound: C1's top generalized eigenvalues are clustered (ratio
    0.995), so both power methods are checked against the dense eigenvalue:
    a Rayleigh quotient never exceeds lambda_max and gets within 1e-3."""
    from oracle.dense import Dense
    G, O, _ = pair(ec, oracle_mod, "c1")
    lam_d = Dense(O).gen_eig()[0].max()
    lam = G.cfl(iters=400, rtol=1e-12)
    assert lam <= lam_d * (1 + 1e-9) and lam >= lam_d * (1 - 1e-3)
    G, O, _ = pair(ec, oracle_mod, "nl16")
    assert G.cfl(iters=300, rtol=1e-12) == pytest.approx(O.power(iters=300, rtol=1e-12), rel=1e-3)


def test_bad_pointer_rejected(ec, oracle_mod):
    import torch
    G, O, _ = pair(ec, oracle_mod, "c1")
    x = torch.zeros(G.n_pad + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(ec.ECError) as e:
        G.apply(ec.OP_KN, x[1:], out=G.zeros())
    assert e.value.code == -1
    with pytest.raises(ec.ECError):
        G.solve(G.zeros(), method=ec.SV_SPE, window=G.window_cap + 1)


# ------------------------------------------------- FP32-refined (FP64 outer)
@pytest.mark.parametrize("name", ["c1", "lshape", "nl16"])
def test_refined_solve(ec, oracle_mod, name):
    """FP32 inner PCG inside the FP64 residual loop: the FP64 residual meets
    rtol; the gauge-invariant flux C x matches the oracle within the
    conditioning bound; the FP32 inner solves add a small gradient part."""
    G, O, _ = pair(ec, oracle_mod, name)
    b = O.kcnT(synth.random_vector(O.n_pad, O.C, 3)) + O.source(2, 1e-3)
    info = G.info(1)
    x = G.solve(G.tensor(b), method=ec.SV_ZERO, rtol=1e-10, precision=ec.PREC_FP32_REFINED,
                inner_rtol=1e-5, inner_maxit=400, outer_max=8, info=info).cpu().numpy()
    I = ec.info_array(info)[0]
    assert I["status"] == 0 and I["rel_res"] <= 1e-10 and I["outer_iters"] >= 2
    nb = np.linalg.norm(b)
    assert np.linalg.norm(b - O.kn(x)) <= 1.5e-10 * nb
    xo, *_ = O.cg(b, rtol=1e-13)
    assert np.linalg.norm(O.curl(x) - O.curl(xo)) <= 1e-8 * np.linalg.norm(O.curl(xo))
    if name != "lshape":
        # cubic cells (scalar Jacobi): the same minimum-norm solution up to the
        # gradient part the FP32 inner solves add; non-cubic cells pick
        # another pseudo-inverse gauge (compared through C x above)
        assert np.linalg.norm(x - xo) <= 1e-5 * np.linalg.norm(xo)
    # b = 0: x = 0, no iterations
    z = G.zeros()
    x0 = G.tensor(xo)
    G.solve(z, x=x0, method=ec.SV_PREV, precision=ec.PREC_FP32_REFINED, info=info)
    I = ec.info_array(info)[0]
    assert I["iters"] == 0 and I["status"] == 0 and not x0.cpu().numpy().any()


def test_refined_trajectory_nonlinear16(ec, oracle_mod):
    """60 SPE steps with FP32-refined solves (rtol 1e-10) against the FP64
    oracle (rtol 1e-12): a_c and the flux within 1e-8."""
    G, O, wl = pair(ec, oracle_mod, "nl16")
    dt = 0.5 * 2 / O.power(iters=60)
    Ao, *_ = O.run(dt, 60, rtol=1e-12)
    A = G.zeros()
    G.set_state(A, rtol=1e-12)
    info = G.info(120)
    G.run(A, 0, 60, dt, ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10,
                                     precision=ec.PREC_FP32_REFINED, inner_rtol=1e-5),
          info=info)
    I = ec.info_array(info)
    assert (I["status"] == 0).all() and (I["rel_res"] <= 1e-10).all()
    got = A.cpu().numpy()
    nrm = np.linalg.norm
    assert nrm((got - Ao)[O.C]) <= 1e-8 * nrm(Ao[O.C])
    assert nrm(O.curl(got) - O.curl(Ao)) <= 1e-8 * nrm(O.curl(Ao))
    assert nrm(got - Ao) <= 1e-5 * nrm(Ao)


def test_refined_graph_replay_equals_eager(ec, oracle_mod):
    G1, O, wl = pair(ec, oracle_mod, "c1")
    dt = 0.9 * 2 / O.power(iters=40)
    kw = dict(rtol=1e-10, precision=ec.PREC_FP32_REFINED, inner_rtol=1e-5, inner_maxit=60,
              outer_max=4)
    opts = ec.step_opts(ec.SV_SPE, window=5, **kw)
    A1 = G1.zeros()
    G1.set_state(A1, rtol=1e-10)
    G1.run(A1, 0, 25, dt, opts)
    G2 = ec.Problem(wl, window_cap=8)
    A2 = G2.zeros()
    G2.set_state(A2, rtol=1e-10)
    G2.run(A2, 0, 10, dt, opts)
    G2.counters_reset()
    g = G2.graph_capture(A2, dt, ec.step_opts(ec.SV_SPE, window=5, graph_iters=(8, 40), **kw))
    for _ in range(15):
        g.launch()
    assert G2.counters()["worst_status"] == 0
    assert np.array_equal(A2.cpu().numpy(), A1.cpu().numpy())


def test_refined_graph_starved_budget_equals_eager(ec, oracle_mod):
    """Captured FP32-refined steps whose inner passes get two iteration
    kernels each: the persistent FP32 tail takes every further iteration of
    every pass, and the trajectory is still the eager one, bit for bit (one
    256-node tile per block on this grid, so the tail's sums are the
    iteration kernel's)."""
    G1, O, wl = pair(ec, oracle_mod, "c1")
    dt = 0.9 * 2 / O.power(iters=40)
    kw = dict(rtol=1e-10, precision=ec.PREC_FP32_REFINED, inner_rtol=1e-5, inner_maxit=60,
              outer_max=4)
    opts = ec.step_opts(ec.SV_SPE, window=5, **kw)
    A1 = G1.zeros()
    G1.set_state(A1, rtol=1e-10)
    info1 = G1.info(2 * 25)
    G1.run(A1, 0, 25, dt, opts, info=info1)
    its = ec.info_array(info1)["iters"][20:]
    assert its.max() > 2                    # the tail has work to do
    G2 = ec.Problem(wl, window_cap=8)
    A2 = G2.zeros()
    G2.set_state(A2, rtol=1e-10)
    G2.run(A2, 0, 10, dt, opts)
    G2.counters_reset()
    g = G2.graph_capture(A2, dt, ec.step_opts(ec.SV_SPE, window=5, graph_iters=(2, 2), **kw))
    for _ in range(15):
        g.launch()
    c = G2.counters()
    assert c["worst_status"] == 0 and c["steps"] == 15
    assert np.array_equal(A2.cpu().numpy(), A1.cpu().numpy())
    # no budget: the first pass issues inner_maxit kernels, later passes one
    # kernel and the tail
    G3 = ec.Problem(wl, window_cap=8)
    A3 = G3.zeros()
    G3.set_state(A3, rtol=1e-10)
    G3.run(A3, 0, 10, dt, opts)
    G3.counters_reset()
    g3 = G3.graph_capture(A3, dt, opts)
    for _ in range(15):
        g3.launch()
    c3 = G3.counters()
    assert c3["worst_status"] == 0 and c3["steps"] == 15
    assert np.array_equal(A3.cpu().numpy(), A1.cpu().numpy())


# ------------------------------------------------ 2.5D (LDS-staged) PCG kernel
@pytest.mark.parametrize("name", ["c1", "lshape", "nl16"])
def test_tiled_pcg_kernel_parity(ec, oracle_mod, name):
    """The 2.5D iteration kernel (forced on small grids, where its column and
    plane chunks overhang the grid) solves to the oracle's solution and gives
    the oracle's trajectory; the refined (FP32 inner) solve uses it too."""
    G, O, wl = pair(ec, oracle_mod, name)
    G.set_pcg_kernel(1)
    b = O.kcnT(synth.random_vector(O.n_pad, O.C, 3)) + O.source(2, 1e-3)
    info = G.info(1)
    x = G.solve(G.tensor(b), method=ec.SV_ZERO, rtol=1e-12, info=info).cpu().numpy()
    assert ec.info_array(info)[0]["status"] == 0
    xo, ito, _, _ = O.cg(b, rtol=1e-12)
    assert np.linalg.norm(b - O.kn(x)) <= 2e-12 * np.linalg.norm(b)
    assert np.linalg.norm(O.curl(x) - O.curl(xo)) <= 1e-10 * np.linalg.norm(O.curl(xo))
    if name == "c1":
        assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
        assert abs(int(ec.info_array(info)[0]["iters"]) - ito) <= max(2, ito // 20)
    xr = G.solve(G.tensor(b), method=ec.SV_ZERO, rtol=1e-10, precision=ec.PREC_FP32_REFINED,
                 info=info).cpu().numpy()
    assert ec.info_array(info)[0]["status"] == 0
    assert np.linalg.norm(b - O.kn(xr)) <= 1.5e-10 * np.linalg.norm(b)
    if name == "nl16":
        dt = 0.5 * 2 / O.power(iters=60)
        Ao, *_ = O.run(dt, 30, rtol=1e-12)
        A = G.zeros()
        G.set_state(A, rtol=1e-12)
        G.run(A, 0, 30, dt, ec.step_opts(ec.SV_SPE, window=8, rtol=1e-12))
        got = A.cpu().numpy()
        assert np.linalg.norm((got - Ao)[O.C]) <= 1e-10 * np.linalg.norm(Ao[O.C])
        assert np.linalg.norm(O.curl(got) - O.curl(Ao)) <= 1e-10 * np.linalg.norm(O.curl(Ao))


def test_tiled_and_node_kernels_agree_at_128(ec, oracle_mod):
    """At 128^3 (where the 2.5D kernel is the default) both kernels reach the
    same solution; the true residual is checked through the oracle's operator."""
    wl = synth.nonlinear(128)
    G = ec.Problem(wl, window_cap=1)
    O = oracle_mod.Problem(wl)
    b = G.tensor(O.kcnT(synth.random_vector(O.n_pad, O.C, 5)))
    xs = []
    for kind in (1, 0):
        G.set_pcg_kernel(kind)
        info = G.info(1)
        xs.append(G.solve(b, method=ec.SV_ZERO, rtol=1e-10, info=info).cpu().numpy())
        assert ec.info_array(info)[0]["status"] == 0
    bn = b.cpu().numpy()
    for x in xs:
        assert np.linalg.norm(bn - O.kn(x)) <= 2e-10 * np.linalg.norm(bn)
    assert np.linalg.norm(xs[0] - xs[1]) <= 1e-8 * np.linalg.norm(xs[1])


def test_pcg_autotuner_cache(ec, oracle_mod, tmp_path):
    """ec_tune_pcg picks a kernel for the grid, records it, and a second
    handle of the same grid gets the recorded pick without timing; solves
    with the tuned kernel still match the oracle."""
    wl = WORKLOADS["nl16"]()
    O = oracle_mod.Problem(wl)
    cache = str(tmp_path / "pcg.txt")
    G = ec.Problem(wl, window_cap=1)
    ti, kb, us = G.tune_pcg(cache)
    assert ti in (0, 16, 32, 64) and us > 0
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("ec-pcg-tiling ")
    G2 = ec.Problem(wl, window_cap=1)
    assert G2.tune_pcg(cache)[:2] == (ti, kb)
    assert len(open(cache).read().splitlines()) == 1
    b = O.kcnT(synth.random_vector(O.n_pad, O.C, 4))
    x = G2.solve(G2.tensor(b), method=ec.SV_ZERO, rtol=1e-12).cpu().numpy()
    xo, *_ = O.cg(b, rtol=1e-12)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
