"""Pins of the FP64 oracle against facts fixed by the mathematics.

Each test checks the oracle against something other than itself: exact
identities of the FIT complex (curl grad = 0, symmetry), closed forms (uniform
fields, diagonal entries, conductivity sums, nullity), a pseudo-inverse by
eigendecomposition, and the closed-form decay of explicit Euler on generalized
eigenvectors of the Schur complement (eqs. 4-8).
"""
import math

import numpy as np
import pytest

import synth
from tests.conftest import small_workload


def cube(N, material=None, J0=1.0e6, wf=synth.WF_SIN):
    mat = material or synth.Material(1.0e6, 0.0, 0.0, synth.NU0)
    return synth.cube_workload(f"c{N}", N, mat, J0, wf)


# --------------------------------------------------------------- FIT complex
@pytest.mark.parametrize("wl_fn", [lambda: cube(6), lambda: small_workload()])
def test_curl_grad_is_exactly_zero(oracle_mod, wl_fn):
    from oracle.dense import gradient
    wl = wl_fn()
    P = oracle_mod.Problem(wl)
    nx, ny, nz = wl.n
    rng = np.random.default_rng(3)
    phi = rng.integers(-1000, 1000, size=(nx + 1) * (ny + 1) * (nz + 1)).astype(float)
    b = P.curl(gradient(wl.n, phi))
    assert np.all(b == 0.0)          # integer arithmetic: exact
    # and K annihilates gradients of potentials vanishing on the boundary
    ph = phi.reshape(nz + 1, ny + 1, nx + 1)
    ph[0], ph[-1] = 0, 0
    ph[:, 0], ph[:, -1] = 0, 0
    ph[:, :, 0], ph[:, :, -1] = 0, 0
    g = gradient(wl.n, ph.ravel())
    assert np.abs(P.apply(g)).max() <= 1e-9 * np.abs(P.apply(np.where(P.D, 0, g + 1))).max()


def test_uniform_field_flux_and_cell_B(oracle_mod):
    """A = B0 x r / 2 has edge integrals whose curl is B0 times the face area."""
    wl = small_workload()
    P = oracle_mod.Problem(wl)
    nx, ny, nz = wl.n
    hx, hy, hz = wl.h
    B0 = np.array([0.3, -0.7, 1.1])
    a = np.zeros(P.n_pad)
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                r = np.array([i * hx, j * hy, k * hz])
                for c, (L, d) in enumerate(((hx, 0), (hy, 1), (hz, 2))):
                    if (c == 0 and i == nx) or (c == 1 and j == ny) or (c == 2 and k == nz):
                        continue
                    mid = r.copy()
                    mid[d] += 0.5 * L
                    A = 0.5 * np.cross(B0, mid)
                    a[synth.edge_slot(wl.n, c, i, j, k)] = A[d] * L
    B = P.cell_B(a)
    assert np.allclose(B, B0[None, :], rtol=0, atol=1e-12)
    b = P.curl(a)
    S = wl.S
    bx = b[:S].reshape(nz + 1, ny + 1, nx + 1)[:nz, :ny, :]
    bz = b[2 * S:].reshape(nz + 1, ny + 1, nx + 1)[:, :ny, :nx]
    assert np.allclose(bx, B0[0] * hy * hz, atol=1e-13)
    assert np.allclose(bz, B0[2] * hx * hy, atol=1e-13)


def test_brauer_reluctivity_on_uniform_field(oracle_mod):
    """In an all-iron box with uniform B0, every cell has nu = k1 e^{k2 B0^2} + k3
    and an interior edge's diagonal of K is 4 nu / h (cube)."""
    N = 6
    k1, k2, k3 = synth.BRAUER
    mat = synth.Material(2e6, k1, k2, k3)
    wl = synth.Workload("iron", (N, N, N), (1.0,) * 3,
                        np.ones(N ** 3, np.uint8), [mat],
                        np.zeros(3 * (N + 1) ** 3))
    P = oracle_mod.Problem(wl)
    h = 1.0 / N
    B0 = 1.3
    a = np.zeros(P.n_pad)   # A = (0, B0 x, 0): a_y(i,j,k) = B0 x_i h
    for k in range(N + 1):
        for j in range(N):
            for i in range(N + 1):
                a[synth.edge_slot(wl.n, 1, i, j, k)] = B0 * (i * h) * h
    nu = P.cell_nu(a)
    nu_exp = k1 * math.exp(k2 * B0 * B0) + k3
    assert np.allclose(nu, nu_exp, rtol=1e-14)
    e = np.zeros(P.n_pad)
    slot = synth.edge_slot(wl.n, 0, 2, 3, 3)
    e[slot] = 1.0
    assert P.apply(e, a)[slot] == pytest.approx(4.0 * nu_exp / h, rel=1e-13)


def test_face_reluctivity_is_mean_of_adjacent_cells(oracle_mod):
    """An edge in the middle of the conductor's top face has two iron|air
    faces, one iron|iron and one air|air face: diag = 2 (nu_i + nu0) / h."""
    N = 12
    k1, k2, k3 = synth.BRAUER
    wl = cube(N, synth.Material(2e6, k1, k2, k3))
    P = oracle_mod.Problem(wl)
    lo, hi = wl.extra["conductor"]
    e = np.zeros(P.n_pad)
    slot = synth.edge_slot(wl.n, 0, lo + 1, lo + 2, hi + 1)   # x-edge on z = top
    assert P.C[slot]
    e[slot] = 1.0
    nu_i = k1 + k3
    h = 1.0 / N
    assert P.apply(e, np.zeros(P.n_pad))[slot] == pytest.approx(2.0 * (nu_i + synth.NU0) / h,
                                                           rel=1e-13)


@pytest.mark.parametrize("wl_fn", [lambda: cube(6), lambda: small_workload()])
def test_K_symmetric_and_psd(oracle_mod, wl_fn):
    from oracle.dense import Dense
    P = oracle_mod.Problem(wl_fn())
    D = Dense(P)
    assert np.max(np.abs(D.K - D.K.T)) <= 1e-12 * np.max(np.abs(D.K))
    w = np.linalg.eigvalsh(D.K)
    assert w.min() > -1e-9 * w.max()


def test_diag_Kn_closed_form(oracle_mod):
    """Every N edge has four air faces: diag K_n = 2 nu0 (h_a/(h_e h_b) + h_b/(h_e h_a))."""
    wl = small_workload()
    P = oracle_mod.Problem(wl)
    hx, hy, hz = wl.h
    nu0 = synth.NU0
    want = [2 * nu0 * (hz / (hx * hy) + hy / (hx * hz)),
            2 * nu0 * (hx / (hy * hz) + hz / (hy * hx)),
            2 * nu0 * (hy / (hz * hx) + hx / (hz * hy))]
    S = wl.S
    e = np.zeros(P.n_pad)
    rng = np.random.default_rng(0)
    for slot in rng.choice(np.flatnonzero(P.N), 60, replace=False):
        e[slot] = 1.0
        assert P.kn(e)[slot] == pytest.approx(want[slot // S], rel=1e-14)
        e[slot] = 0.0
    # cube: 4 nu0 / h
    P2 = oracle_mod.Problem(cube(8))
    e = np.zeros(P2.n_pad)
    slot = np.flatnonzero(P2.N)[17]
    e[slot] = 1.0
    assert P2.kn(e)[slot] == pytest.approx(4 * nu0 * 8, rel=1e-14)


@pytest.mark.parametrize("N,Nc", [(6, 2), (8, 2), (12, 4)])
def test_nullity_of_Kn(oracle_mod, N, Nc):
    """dim null(K_n) = interior air nodes + 1 (floating conductor potential)
    = (N-1)^3 - (Nc+1)^3 + 1; K_n is PSD."""
    from oracle.dense import Dense
    P = oracle_mod.Problem(cube(N))
    lo, hi = synth.conductor_range(N)
    assert hi - lo + 1 == Nc
    D = Dense(P)
    w = np.linalg.eigvalsh(D.Kn)
    assert w.min() > -1e-9 * w.max()
    null = int(np.count_nonzero(w < 1e-9 * w.max()))
    assert null == (N - 1) ** 3 - (Nc + 1) ** 3 + 1


def test_edge_counts_c1(oracle_mod):
    P = oracle_mod.Problem(synth.linear_c1(12))
    assert (P.C.sum(), P.N.sum()) == (300, 4056)
    P = oracle_mod.Problem(synth.nonlinear(48))
    assert (P.C.sum(), P.N.sum()) == (13872, 304224)


def test_conductivity_sum(oracle_mod):
    """sum_e M_sigma,e h_e^2 = 3 sigma V_conductor (each cell spreads its
    sigma V over its 12 edges, a quarter each)."""
    wl = small_workload(material=synth.Material(3.5e6))
    P = oracle_mod.Problem(wl)
    hx, hy, hz = wl.h
    S = wl.S
    hh = np.concatenate([np.full(S, hx * hx), np.full(S, hy * hy), np.full(S, hz * hz)])
    ncell = int(np.count_nonzero(wl.cell_mat))
    assert (P.msig * hh).sum() == pytest.approx(3 * 3.5e6 * ncell * hx * hy * hz, rel=1e-13)


def test_coil_divergence_free():
    from oracle.dense import divergence
    for N in (6, 12, 16, 22, 48):
        wl = synth.linear_c1(N)
        assert np.abs(divergence(wl.n, wl.edge_current)).max() == 0.0
    # total current through a half plane x = const equals J0 (2h)^2 at N=12
    wl = synth.linear_c1(12)
    h = 1 / 12
    tot = sum(wl.edge_current[synth.edge_slot(wl.n, 1, 1, 5, k)] +
              wl.edge_current[synth.edge_slot(wl.n, 1, 2, 5, k)] +
              wl.edge_current[synth.edge_slot(wl.n, 1, 3, 5, k)] for k in range(13))
    assert tot == pytest.approx(-1e6 * (2 * h) ** 2, rel=1e-14)


# ------------------------------------------------------------------- solver
@pytest.mark.parametrize("wl_fn", [lambda: cube(6), lambda: cube(8), lambda: small_workload()])
def test_cg_equals_moore_penrose(oracle_mod, wl_fn):
    """Weak gauging (Sec. II): CG from zero on the consistent singular system
    returns the minimum-norm solution K_n^+ b of the eigendecomposition."""
    from oracle.dense import Dense
    wl = wl_fn()
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    Kp, Vnull = D.pinv_kn()
    for b in (P.source(1, 1e-3) if wl.edge_current.any() else None,
              P.kcnT(synth.random_vector(P.n_pad, P.C, 5))):
        if b is None or not b.any():
            continue
        bn = b[D.n_slots]
        assert np.linalg.norm(Vnull.T @ bn) <= 1e-12 * np.linalg.norm(bn)   # consistent
        x, it, rel, st = P.cg(b, rtol=1e-13)
        assert st == 0 and rel <= 1e-13
        xd = Kp @ bn
        assert np.linalg.norm(x[D.n_slots] - xd) <= 1e-10 * np.linalg.norm(xd)
        assert np.linalg.norm(Vnull.T @ x[D.n_slots]) <= 1e-10 * np.linalg.norm(xd)
        assert np.all(x[~P.N] == 0.0)


def test_cg_zero_rhs_and_maxit(oracle_mod):
    P = oracle_mod.Problem(cube(6))
    x, it, rel, st = P.cg(np.zeros(P.n_pad), x0=np.ones(P.n_pad))
    assert it == 0 and st == 0 and not x.any()
    _, it, _, st = P.cg(P.source(1, 1e-3), maxit=1, rtol=1e-14)
    assert st == -3 and it == 1


# ------------------------------------------------------- time integration
def _state_from_ac(P, ac):
    """Full state (a_c, a_n) and s_c = K_n^+ K_cn^T a_c for a given a_c."""
    A = np.where(P.C, ac, 0.0)
    sc, *_ = P.cg(P.kcnT(A), rtol=1e-14)
    A = A - sc
    A[P.C] = ac[P.C]
    return A, sc


def test_closed_form_decay_and_sign(oracle_mod):
    """j = 0, a_c^0 = v_i (K_S v = lambda M_c v): explicit Euler gives
    a_c^m = (1 - dt lambda)^m v_i exactly (eq. 6 with the sign of eq. 5a)."""
    from oracle.dense import Dense
    wl = cube(6)
    wl.amp = 0.0
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    lam, V = D.gen_eig()
    dt = 0.9 * 2 / lam.max()
    for idx in (0, len(lam) // 2, len(lam) - 1):
        ac = np.zeros(P.n_pad)
        ac[D.c_slots] = V[:, idx] / np.abs(V[:, idx]).max()
        A, sc = _state_from_ac(P, ac)
        M = 7
        A2, _, rec, *_ = P.run(dt, M, rtol=1e-14, A=A, sc=sc, rec_every=1)
        for m in range(1, M + 1):
            want = (1 - dt * lam[idx]) ** m * ac[D.c_slots]
            got = rec[m - 1][D.c_slots]
            assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(ac) + 1e-300


def test_cfl_bound_sharp_and_power_method(oracle_mod):
    """Eq. (8): dt = 0.99 * 2/lam_max decays, 1.01 * 2/lam_max grows by
    |1 - dt lam_max| per step; the power method finds lam_max."""
    from oracle.dense import Dense
    wl = cube(6)
    wl.amp = 0.0
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    lam, V = D.gen_eig()
    lmax = lam.max()
    assert P.power(iters=300) == pytest.approx(lmax, rel=1e-6)
    ac = np.zeros(P.n_pad)
    ac[D.c_slots] = V[:, -1]
    A, sc = _state_from_ac(P, ac)
    for f, grows in ((0.99, False), (1.01, True)):
        dt = f * 2 / lmax
        A2, *_ = P.run(dt, 20, rtol=1e-14, A=A, sc=sc)
        ratio = np.linalg.norm(A2[D.c_slots]) / np.linalg.norm(ac[D.c_slots])
        assert ratio == pytest.approx(abs(1 - dt * lmax) ** 20, rel=1e-6)
        assert (ratio > 1) == grows


def test_dense_recursion_trajectory(oracle_mod):
    """The oracle's CG-based steps equal the dense recursion with the exact
    pseudo-inverse (eqs. 6, 7) on a tiny grid with the sine source."""
    from oracle.dense import Dense
    wl = small_workload(amp=3.0e3, freq=50.0)
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    Kp, _ = D.pinv_kn()
    lam, _ = D.gen_eig()
    dt = 0.8 * 2 / lam.max()
    M = 25
    _, _, rec, *_ = P.run(dt, M, rtol=1e-14, rec_every=1)
    ac = np.zeros(len(D.ic))
    for m in range(1, M + 1):
        j = P.source(m, dt)[D.n_slots]
        ac = ac - dt / D.Mc * (D.Kc @ ac + D.Kcn @ (Kp @ (j - D.Kcn.T @ ac)))
        an = Kp @ (j - D.Kcn.T @ ac)
        want = np.concatenate([ac, an])
        got = np.concatenate([rec[m - 1][D.c_slots], rec[m - 1][D.n_slots]])
        assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


def test_static_fixed_point(oracle_mod):
    """With a DC source the fixed point of eqs. (6)-(7) carries the B field of
    the full magnetostatic system K a = j; one step leaves it unchanged."""
    from oracle.dense import Dense
    wl = small_workload(waveform=synth.WF_DC, amp=1.0e3)
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    Kp, _ = D.pinv_kn()
    j = P.source(1, 1.0)[D.n_slots]
    KS = D.schur()
    ac = np.linalg.lstsq(KS, -D.Kcn @ (Kp @ j), rcond=1e-12)[0]
    an = Kp @ (j - D.Kcn.T @ ac)
    A = np.zeros(P.n_pad)
    A[D.c_slots], A[D.n_slots] = ac, an
    rhs = np.zeros(len(D.idx))
    rhs[D.inn] = j
    af = np.linalg.lstsq(D.K, rhs, rcond=1e-12)[0]
    Afull = np.zeros(P.n_pad)
    Afull[D.idx] = af
    bA, bF = P.curl(A), P.curl(Afull)
    assert np.linalg.norm(bA - bF) <= 1e-8 * np.linalg.norm(bF)
    _, sc = _state_from_ac(P, A)
    lam, _ = D.gen_eig()
    A2, *_ = P.run(0.5 * 2 / lam.max(), 1, rtol=1e-14, A=A, sc=sc)
    assert np.linalg.norm(A2[D.c_slots] - ac) <= 1e-9 * np.linalg.norm(ac)


def test_energy_non_increasing(oracle_mod):
    """Linear, j = 0, dt below the bound: 1/2 a_c^T K_S a_c never grows."""
    from oracle.dense import Dense
    wl = cube(6)
    wl.amp = 0.0
    P = oracle_mod.Problem(wl)
    D = Dense(P)
    KS = D.schur()
    lam, _ = D.gen_eig()
    ac = synth.random_vector(P.n_pad, P.C, 11)
    A, sc = _state_from_ac(P, ac)
    _, _, rec, *_ = P.run(0.95 * 2 / lam.max(), 30, rtol=1e-13, A=A, sc=sc, rec_every=1)
    E = [0.5 * r[D.c_slots] @ KS @ r[D.c_slots] for r in rec]
    assert all(E[i + 1] <= E[i] * (1 + 1e-12) for i in range(len(E) - 1))


def test_waveforms(oracle_mod):
    L = oracle_mod.lib()
    assert L.or_waveform(1, 2.0, 50.0, 0.5, 1, 3, 1e-3) == pytest.approx(2 * math.sin(2 * math.pi * 50 * 3e-3))
    assert L.or_waveform(2, 2.0, 0.0, 0.5, 1000, 250, 1e-3) == pytest.approx(0.5)
    assert L.or_waveform(2, 2.0, 0.0, 0.5, 1000, 2500, 1e-3) == 2.0
    assert L.or_waveform(3, 1.0, 0.0, 0.5, 1, 120, 1e-3) == pytest.approx(1 - math.exp(-0.24))
    assert L.or_waveform(0, 1.5, 0.0, 0.5, 1, 7, 1e-3) == 1.5
