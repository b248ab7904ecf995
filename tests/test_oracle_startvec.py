"""Pins of the SPE / POD start-vector oracle (eqs. 10-14)."""
import numpy as np
import pytest

import synth
from tests.conftest import small_workload


@pytest.fixture(scope="module")
def setup(oracle_mod):
    wl = synth.linear_c1(12)
    P = oracle_mod.Problem(wl)
    lam = P.power(iters=40)
    dt = 0.9 * 2 / lam
    # a window of consecutive CPL solutions (range-space, nearly parallel)
    A = np.zeros(P.n_pad)
    sc = np.zeros(P.n_pad)
    sols = []
    for m in range(1, 12):
        A, sc, *_ = P.run(dt, 1, rtol=1e-13, A=A, sc=sc, m0=m - 1)
        sols.append(sc.copy())
    return P, dt, sols


def dense_projection(P, X, b):
    """x0 of eq. (10) through a Householder QR (numpy) instead of MGS."""
    Q, R = np.linalg.qr(np.column_stack(X))
    keep = np.abs(np.diag(R)) > 1e-10 * np.abs(R).max()
    Q = Q[:, keep]
    KQ = np.column_stack([P.kn(q) for q in Q.T])
    return Q @ np.linalg.solve(Q.T @ KQ, Q.T @ b)


def test_spe_galerkin_orthogonality_and_qr_equivalence(setup):
    from oracle.startvec import mgs_basis, spe_start
    P, dt, sols = setup
    X = sols[-6:-1]
    b = P.kcnT(synth.random_vector(P.n_pad, P.C, 7))
    x0 = spe_start(P, X, b)
    U = np.column_stack(mgs_basis(X))
    assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-12
    r = b - P.kn(x0)
    assert np.linalg.norm(U.T @ r) <= 1e-10 * np.linalg.norm(b)
    rng = np.random.default_rng(1)
    Xw = [P.kn(synth.random_vector(P.n_pad, P.N, s)) for s in range(5)]
    assert np.allclose(spe_start(P, Xw, b), dense_projection(P, Xw, b), rtol=0,
                       atol=1e-10 * np.linalg.norm(dense_projection(P, Xw, b)))


def test_spe_exact_when_solution_in_span(setup):
    """b in K_n span(X): the projection returns the solution itself."""
    from oracle.startvec import spe_start
    P, dt, sols = setup
    X = sols[-5:]
    c = np.array([0.3, -1.0, 2.0, 0.5, 1.5])
    x = np.column_stack(X) @ c
    x0 = spe_start(P, X, P.kn(x))
    assert np.linalg.norm(x0 - x) <= 1e-6 * np.linalg.norm(x)   # nearly parallel window
    Xw = [synth.random_vector(P.n_pad, P.N, 40 + s) for s in range(4)]
    Xw = [P.kn(v) for v in Xw]
    x = Xw[0] - 2 * Xw[3]
    assert np.linalg.norm(spe_start(P, Xw, P.kn(x)) - x) <= 1e-11 * np.linalg.norm(x)


def test_mgs_drops_dependent_columns(setup):
    from oracle.startvec import mgs_basis
    P, _, sols = setup
    X = [sols[0], 2.0 * sols[0], sols[1], sols[0] - sols[1]]
    assert len(mgs_basis(X)) == 2


def test_pod_untruncated_equals_spe(setup):
    """With every mode kept, U_POD spans the window: eq. (14) = eq. (10)."""
    from oracle.startvec import pod_start, spe_start
    P, _, _ = setup
    Xw = [P.kn(synth.random_vector(P.n_pad, P.N, 70 + s)) for s in range(6)]
    b = P.kcnT(synth.random_vector(P.n_pad, P.C, 8))
    x_pod, k, info = pod_start(P, Xw, b, eps=0.0)
    assert k == 6 and info == pytest.approx(1.0)
    x_spe = spe_start(P, Xw, b)
    assert np.linalg.norm(x_pod - x_spe) <= 1e-10 * np.linalg.norm(x_spe)


def test_pod_truncation_and_information(setup):
    from oracle.startvec import pod_basis
    P, _, sols = setup
    X = sols[-10:]
    U, k, info, s = pod_basis(X, eps=1e-4, kmax=None)
    assert k == int(np.sum(s >= 1e-4 * s[0]))
    assert 1 <= k < 10
    assert info == pytest.approx(s[:k].sum() / s.sum())
    assert 0.99 < info <= 1.0
    # method of snapshots: sqrt(eig(X^T X)) are the singular values
    Xm = np.column_stack(X)
    ev = np.sort(np.linalg.eigvalsh(Xm.T @ Xm))[::-1]
    assert np.allclose(np.sqrt(np.clip(ev[:k], 0, None)), s[:k], rtol=1e-8)
    U2, k2, _, _ = pod_basis(X, eps=1e-4, kmax=3)
    assert k2 == min(3, k)


def test_spe_start_reduces_iterations(setup):
    """The start vector is at least as good as the previous solution (it lies in
    the window's span and minimises the K_n-energy error there)."""
    from oracle.startvec import spe_start
    P, dt, sols = setup
    A = np.zeros(P.n_pad)
    b_next = None
    # rebuild the next CPL right-hand side from the oracle state after 11 steps
    A = np.zeros(P.n_pad); sc = np.zeros(P.n_pad)
    A, sc, *_ = P.run(dt, 11, rtol=1e-13, A=A, sc=sc)
    A2, sc2, *_ = P.run(dt, 1, rtol=1e-13, A=A.copy(), sc=sc.copy(), m0=11)
    b_next = P.kcnT(A2)
    x_true = sc2
    x_spe = spe_start(P, sols[-5:], b_next)
    e_spe = x_true - x_spe
    e_prev = x_true - sols[-1]
    assert e_spe @ P.kn(e_spe) <= e_prev @ P.kn(e_prev) * (1 + 1e-9)
    _, it_spe, _, _ = P.cg(b_next, x0=x_spe, rtol=1e-8)
    _, it_zero, _, _ = P.cg(b_next, rtol=1e-8)
    assert it_spe < it_zero


def test_gauge_rows_closed_form_and_range_space(setup):
    """D G delta_v is the 7-point graph Laplacian (6 at a free node v, -1 at
    its free neighbours); D vanishes on range(K_n) and on the minimum-norm
    solutions, which are orthogonal to every gradient."""
    from oracle.dense import gradient
    from oracle.startvec import free_nodes, gauge_rows
    P, dt, sols = setup
    nx, ny, nz = P.wl.n
    S = (nx + 1) * (ny + 1) * (nz + 1)
    free = free_nodes(P)
    node = lambda i, j, k: (k * (ny + 1) + j) * (nx + 1) + i
    v = node(2, 3, 2)
    assert free[v] and not free[node(0, 3, 2)]
    phi = np.zeros(S)
    phi[v] = 1.0
    g = gradient(P.wl.n, phi)
    assert not g[~P.N].any() and np.abs(P.kn(g)).max() < 1e-9 * np.abs(P.kn(sols[-1])).max()
    full = np.zeros(S)
    full[free] = gauge_rows(P, g, free)
    assert full[v] == 6.0
    for w in (node(1, 3, 2), node(3, 3, 2), node(2, 2, 2), node(2, 4, 2), node(2, 3, 1),
              node(2, 3, 3)):
        assert full[w] == (-1.0 if free[w] else 0.0)
    assert np.abs(full).sum() == 6.0 + free[[node(1, 3, 2), node(3, 3, 2), node(2, 2, 2),
                                              node(2, 4, 2), node(2, 3, 1), node(2, 3, 3)]].sum()
    for x in sols[-3:] + [P.kn(synth.random_vector(P.n_pad, P.N, 5))]:
        # each entry is a sum of six edge values of size up to max|x|
        assert np.abs(gauge_rows(P, x, free)).max() <= 1e-10 * np.abs(x).max()


def test_gauge_eta_is_half_the_kn_diagonal(setup):
    from oracle.startvec import gauge_eta
    P, dt, sols = setup
    nx, ny, nz = P.wl.n
    S = (nx + 1) * (ny + 1) * (nz + 1)
    for c in range(3):
        e = np.zeros(P.n_pad)
        slot = c * S + (2 * (ny + 1) + 2) * (nx + 1) + 1     # an edge far from the iron
        assert P.N[slot]
        e[slot] = 1.0
        assert gauge_eta(P) == pytest.approx(0.5 * P.kn(e)[slot], rel=1e-14)


def test_gauge_penalty_removes_null_directions(setup):
    """Window = {x*, gradient}: the projection of eq. (10) is singular (the
    gradient has no K_n energy); with the penalty it returns x* itself.  On a
    window inside range(K_n) the penalty changes nothing."""
    from oracle.dense import gradient
    from oracle.startvec import free_nodes, mgs_basis, spe_start
    P, dt, sols = setup
    nx, ny, nz = P.wl.n
    S = (nx + 1) * (ny + 1) * (nz + 1)
    rng = np.random.default_rng(3)
    phi = np.where(free_nodes(P), rng.standard_normal(S), 0.0)
    g = gradient(P.wl.n, phi)
    xs = sols[-1]
    b = P.kn(xs)
    U = np.column_stack(mgs_basis([xs, g]))
    H = U.T @ np.column_stack([P.kn(u) for u in U.T])
    assert np.linalg.cond(H) > 1e10
    x0 = spe_start(P, [xs, g], b)
    assert np.linalg.norm(x0 - xs) <= 1e-10 * np.linalg.norm(xs)
    X = sols[-6:-1]
    bb = P.kcnT(synth.random_vector(P.n_pad, P.C, 8))
    a, z = spe_start(P, X, bb, penalty=1.0), spe_start(P, X, bb, penalty=0.0)
    assert np.linalg.norm(a - z) <= 1e-8 * np.linalg.norm(z)
