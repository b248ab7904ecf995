"""The allocation-free PCG solve (ec_solve_static: scratch in the library's
static device array) against ec_solve on the same inputs: two calls in a
row, the second on a smaller grid, then a grid beyond the array's limit."""
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


def test_static_solve_equals_solve(ec, oracle_mod):
    for wl in (synth.nonlinear(48), synth.linear_c1(12)):      # the second one smaller
        O = oracle_mod.Problem(wl)
        G = ec.Problem(wl, window_cap=1)
        bh = O.kcnT(synth.random_vector(O.n_pad, O.C, 17)) + O.source(3, 1e-4)
        b = G.tensor(bh)
        xs, *_ = O.cg(bh, rtol=1e-3)            # a rough start for PREV
        for method in (ec.SV_ZERO, ec.SV_PREV):
            x0 = G.tensor(xs)
            i1, i2 = G.info(1), G.info(1)
            x1 = G.solve(b, x=x0.clone(), method=method, rtol=1e-10, info=i1)
            x2 = G.solve_static(b, x=x0.clone(), method=method, rtol=1e-10, info=i2)
            r1, r2 = ec.info_array(i1)[0], ec.info_array(i2)[0]
            assert r1["status"] == 0 and r2["status"] == 0
            assert r1["iters"] == r2["iters"] and r1["rel_res"] == r2["rel_res"]
            assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy()), (wl.name, method)
            if method == ec.SV_ZERO:
                xo, *_ = O.cg(b.cpu().numpy(), rtol=1e-12)
                assert (np.linalg.norm(x2.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo))
        G.close()


def test_static_solve_rejects(ec):
    G = ec.Problem(synth.linear_c1(12), window_cap=1)
    b = G.zeros()
    with pytest.raises(ec.ECError) as ei:
        G.solve_static(b, method=ec.SV_SPE)
    assert ei.value.code == ec.EC_ERR_ARG
    with pytest.raises(ec.ECError) as ei:
        G.solve_static(b, precision=ec.PREC_FP32_REFINED)
    assert ei.value.code == ec.EC_ERR_ARG
    G.close()
    big = ec.Problem(synth.nonlinear(80), window_cap=1)     # n_padded 1,594,323
    assert big.n_pad > ec.STATIC_MAX_NPAD
    with pytest.raises(ec.ECError) as ei:
        big.solve_static(big.zeros())
    assert ei.value.code == ec.EC_ERR_ARG
    big.close()
