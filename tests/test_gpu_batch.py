"""Batched stepping of uneven instances (C-ABI ec_batch_*): a batched
instance equals the same problem stepped alone (bitwise), graph replay equals
eager, parity with the oracle, and the autotuner's cache."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ec():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06721_amd as ec
    return ec


def instances(count=4, seed=7, sizes=(8, 11, 14, 17)):
    """Uneven instances in the manner of the multi-query batch draws:
    conductivity 10^U(5,7), Brauer coefficients within 10 %."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = sizes[i % len(sizes)]
        sigma = 10.0 ** rng.uniform(5.0, 7.0)
        ks = [b * (1.0 + rng.uniform(-0.1, 0.1)) for b in synth.BRAUER]
        out.append(synth.nonlinear(N, ramp_steps=20, J0=6.0e6, sigma=sigma, brauer=tuple(ks),
                                   name=f"inst{i}_N{N}"))
    return out


def make_batch(ec, wls, stream):
    import torch
    probs = [ec.Problem(w, window_cap=8, stream=stream) for w in wls]
    return probs, ec.Batch(probs)


def test_batch_equals_single(ec, oracle_mod):
    import torch
    wls = instances()
    dts = [0.5 * 2 / oracle_mod.Problem(w).power(iters=40) for w in wls]
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10)
    s = torch.cuda.Stream()
    probs, B = make_batch(ec, wls, s)
    As = [p.zeros() for p in probs]
    for p, A in zip(probs, As):
        p.set_state(A, rtol=1e-10)
    B.run(0, 25, dts, As, opts)
    for w, dt, A, p in zip(wls, dts, As, probs):
        G = ec.Problem(w, window_cap=8)
        A1 = G.zeros()
        G.set_state(A1, rtol=1e-10)
        G.run(A1, 0, 25, dt, opts)
        assert np.array_equal(A.cpu().numpy(), A1.cpu().numpy()), w.name
        c, c1 = p.counters(), G.counters()
        assert c["iters_src"] == c1["iters_src"] and c["iters_cpl"] == c1["iters_cpl"]
        assert c["worst_status"] == 0 and c["steps"] == 25


def test_batch_parity_with_oracle(ec, oracle_mod):
    import torch
    wls = instances(count=2, sizes=(10, 13))
    Os = [oracle_mod.Problem(w) for w in wls]
    dts = [0.5 * 2 / O.power(iters=40) for O in Os]
    s = torch.cuda.Stream()
    probs, B = make_batch(ec, wls, s)
    As = [p.zeros() for p in probs]
    for p, A in zip(probs, As):
        p.set_state(A, rtol=1e-12)
    B.run(0, 20, dts, As, ec.step_opts(ec.SV_ZERO, rtol=1e-12))
    for O, dt, A in zip(Os, dts, As):
        Ao, *_ = O.run(dt, 20, rtol=1e-12)
        got = A.cpu().numpy()
        assert np.linalg.norm(got - Ao) <= 1e-10 * np.linalg.norm(Ao)


def test_batch_graph_equals_eager(ec, oracle_mod):
    import torch
    wls = instances()
    dts = [0.5 * 2 / oracle_mod.Problem(w).power(iters=40) for w in wls]
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10)
    runs = []
    for graph in (False, True):
        s = torch.cuda.Stream()
        probs, B = make_batch(ec, wls, s)
        As = [p.zeros() for p in probs]
        for p, A in zip(probs, As):
            p.set_state(A, rtol=1e-10)
        B.run(0, 10, dts, As, opts)
        if graph:
            g = B.graph_capture(dts, As, ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10,
                                                      graph_iters=(4, 300)))
            for _ in range(12):
                g.launch()
            del g
        else:
            B.run(-1, 12, dts, As, opts)
        runs.append([A.cpu().numpy() for A in As])
        assert all(p.counters()["worst_status"] == 0 for p in probs)
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("tiles", [1, 4])
def test_batch_graph_starved_budget_equals_eager(ec, oracle_mod, tiles):
    """Captured batch steps whose solves get one or two iteration launches:
    the persistent batched tail runs every further iteration of every
    instance, and the trajectories are the eager ones bit for bit (one tile
    per block, and several tiles per block)."""
    import torch
    wls = instances()
    dts = [0.5 * 2 / oracle_mod.Problem(w).power(iters=40) for w in wls]
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10)
    runs = []
    for budget in (None, (1, 2), (2, 1)):
        s = torch.cuda.Stream()
        probs, B = make_batch(ec, wls, s)
        B.set_tiles(tiles)
        As = [p.zeros() for p in probs]
        for p, A in zip(probs, As):
            p.set_state(A, rtol=1e-10)
        B.run(0, 6, dts, As, opts)
        for p in probs:
            p.counters_reset()
        if budget is None:
            B.run(-1, 10, dts, As, opts)
        else:
            g = B.graph_capture(dts, As, ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10,
                                                      graph_iters=budget))
            for _ in range(10):
                g.launch()
            g.close()
        cs = [p.counters() for p in probs]
        assert all(c["worst_status"] == 0 and c["steps"] == 10 for c in cs)
        runs.append(([A.cpu().numpy() for A in As],
                     [(c["iters_src"], c["iters_cpl"]) for c in cs]))
        B.close()
        for p in probs:
            p.close()
    for r in runs[1:]:
        assert r[1] == runs[0][1]
        for a, b in zip(r[0], runs[0][0]):
            assert np.array_equal(a, b)


def test_batch_autotune_cache(ec, oracle_mod, tmp_path):
    import torch
    wls = instances(count=3)
    dts = [0.5 * 2 / oracle_mod.Problem(w).power(iters=40) for w in wls]
    cache = str(tmp_path / "tiles.txt")
    s = torch.cuda.Stream()
    probs, B = make_batch(ec, wls, s)
    f, us = B.autotune(cache)
    assert f in (1, 2, 4, 8) and us > 0
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("ec-batch-tiles ")
    # the same shapes: the cached pick, no new line
    probs2, B2 = make_batch(ec, wls, torch.cuda.Stream())
    f2, us2 = B2.autotune(cache)
    assert (f2, us2) == (f, pytest.approx(us, rel=1e-3))
    assert len(open(cache).read().splitlines()) == 1
    # stepping with the tuned grids still matches the oracle
    As = [p.zeros() for p in probs2]
    for p, A in zip(probs2, As):
        p.set_state(A, rtol=1e-12)
    B2.set_tiles(4)
    B2.run(0, 8, dts, As, ec.step_opts(ec.SV_ZERO, rtol=1e-12))
    for w, dt, A in zip(wls, dts, As):
        Ao, *_ = oracle_mod.Problem(w).run(dt, 8, rtol=1e-12)
        assert np.linalg.norm(A.cpu().numpy() - Ao) <= 1e-10 * np.linalg.norm(Ao)


def test_batch_errors(ec):
    import torch
    wls = instances(count=2)
    a = ec.Problem(wls[0], window_cap=4)          # own streams
    b = ec.Problem(wls[1], window_cap=4)
    with pytest.raises(ValueError):
        ec.Batch([a, b])
    s = torch.cuda.Stream()
    probs, B = make_batch(ec, wls, s)
    As = [p.zeros() for p in probs]
    with pytest.raises(ec.ECError):               # FP32-refined is not batched
        B.step([1e-6, 1e-6], As, ec.step_opts(ec.SV_ZERO, precision=ec.PREC_FP32_REFINED))
    with pytest.raises(ec.ECError):
        B.set_tiles(0)
