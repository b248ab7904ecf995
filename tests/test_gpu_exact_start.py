"""A solve whose SPE or POD start already meets the tolerance ends in the PCG
init kernel: the start combination's own sums of r0^2 and b^2 take the first
iteration's stop decision (eq. 10 / eq. 14 starts, Sec. III).  The record
shows zero iterations and the start's residual, the solution is the start
vector, and the following iteration and tail kernels only pass the record
on; eagerly, in a captured step, and in a batch."""
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


@pytest.mark.parametrize("method", ["spe", "pod"])
def test_exact_start_stops_in_init(ec, oracle_mod, method):
    # cubic cells: one Jacobi diagonal on every nonconducting edge, so the
    # zero-start PCG solution carries no gradient part and the grad-div
    # weighted SPE projection reproduces 2 x1 (on non-cubic cells it weighs
    # the gradient part that Jacobi-PCG leaves and the start is not exact)
    wl = synth.linear_c1(12)
    O = oracle_mod.Problem(wl)
    G = ec.Problem(wl, window_cap=8)
    meth = ec.SV_SPE if method == "spe" else ec.SV_POD
    seq = ec.SEQ_ADJ
    G.history_reset(seq)
    b = O.source(1, 1e-3) + O.kcnT(synth.random_vector(O.n_pad, O.C, 5))
    # first solve: empty history, PCG from zero to 1e-12; its solution is pushed
    info = G.info(1)
    x1 = G.solve(G.tensor(b), seq=seq, method=meth, window=4, info=info, rtol=1e-12)
    I1 = ec.info_array(info)[0]
    assert I1["status"] == 0 and I1["iters"] > 0
    # second solve of 2 b at 1e-8: the start 2 x1 leaves ~1e-12 and ends the solve
    info = G.info(1)
    x2 = G.solve(G.tensor(2.0 * b), seq=seq, method=meth, window=4, info=info, rtol=1e-8)
    I2 = ec.info_array(info)[0]
    assert I2["status"] == 0
    assert I2["iters"] == 0
    assert I2["rel_res"] <= 1e-8
    assert I2["r0_rel"] == I2["rel_res"]          # no iteration ran after the start
    x1n, x2n = x1.cpu().numpy(), x2.cpu().numpy()
    # the start's residual as the oracle computes it, and the solution
    r = 2.0 * b - O.kn(np.where(O.N, x2n, 0.0))
    assert abs(np.linalg.norm(r) / np.linalg.norm(2.0 * b) - I2["rel_res"]) <= 1e-13
    kx = O.kn(np.where(O.N, x2n, 0.0))
    assert np.linalg.norm(kx - 2.0 * b) <= 1e-10 * np.linalg.norm(2.0 * b)
    assert np.linalg.norm(x2n - 2.0 * x1n) <= 1e-9 * np.linalg.norm(x1n)
    G.close()


def test_source_solves_stop_in_init_eager_and_captured(ec, oracle_mod):
    """The source right-hand side keeps its shape over the run: from the
    third step on every source solve ends on its start vector, in eager steps
    and in graph replays alike (and the replays equal the eager run)."""
    wl = synth.nonlinear(16, ramp_steps=40, J0=6.0e6)
    O = oracle_mod.Problem(wl)
    dt = 0.5 * 2 / O.power(iters=40)
    runs = []
    for captured in (False, True):
        G = ec.Problem(wl, window_cap=8)
        A = G.zeros()
        G.set_state(A, rtol=1e-10)
        opts = ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10)
        info = G.info(2 * 6)
        G.run(A, 0, 6, dt, opts, info=info)
        I = ec.info_array(info)
        assert (I["status"] == 0).all()
        assert (I[0::2]["iters"][2:] == 0).all()
        G.counters_reset()
        if captured:
            g = G.graph_capture(A, dt, ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10,
                                                    graph_iters=(2, 16)))
            for _ in range(8):
                g.launch()
            g.close()
        else:
            G.run(A, 6, 8, dt, opts)
        c = G.counters()
        assert c["worst_status"] == 0 and c["steps"] == 8
        assert c["iters_src"] == 0
        runs.append((A.cpu().numpy(), c["iters_cpl"]))
        G.close()
    assert runs[0][1] == runs[1][1]
    assert np.array_equal(runs[0][0], runs[1][0])


def test_batch_source_solves_stop_in_init(ec, oracle_mod):
    """Batched instances: the source solves end in the batched init too."""
    import torch
    wls = [synth.nonlinear(n, ramp_steps=40, J0=6.0e6) for n in (12, 16)]
    dts = [0.5 * 2 / oracle_mod.Problem(w).power(iters=40) for w in wls]
    s = torch.cuda.Stream()
    probs = [ec.Problem(w, window_cap=8, stream=s) for w in wls]
    B = ec.Batch(probs)
    As = [p.zeros() for p in probs]
    for p, A in zip(probs, As):
        p.set_state(A, rtol=1e-10)
    opts = ec.step_opts(ec.SV_SPE, window=8, rtol=1e-10)
    B.run(0, 4, dts, As, opts)
    for p in probs:
        p.counters_reset()
    B.run(4, 6, dts, As, opts)
    for p in probs:
        c = p.counters()
        assert c["worst_status"] == 0 and c["steps"] == 6
        assert c["iters_src"] == 0 and c["iters_cpl"] > 0
    B.close()
    for p in probs:
        p.close()
