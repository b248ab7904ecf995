"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-side assembly validates inputs and agrees with
the oracle's independent edge classification."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from tests.conftest import ROOT, small_workload

HEADER = os.path.join(ROOT, "include", "ec.h")


@pytest.fixture(scope="module")
def L():
    from paper_1611_06721_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libec.so not built (run __graft_entry__.build())")
    return _lib.load()


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ec_[a-z_0-9]+)\s*\(", txt)))


def test_header_symbols_exported(L):
    from paper_1611_06721_amd import _lib
    syms = declared_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(L, s), f"{s} not exported"
    assert set(syms) == set(_lib.SIGNATURES), "binding signatures out of sync with ec.h"


def test_roctx_phase_ranges_linked(L):
    """The library marks its host phases (step, solves, start vector, PCG,
    update, pushes) as roctx ranges: it imports the push/pop pair from the
    roctx library rather than carrying its own stubs."""
    import shutil
    import subprocess
    from paper_1611_06721_amd import _lib
    nm = shutil.which("nm")
    if not nm:
        pytest.skip("nm not installed")
    out = subprocess.run([nm, "-D", "--undefined-only", _lib.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    assert re.search(r"\bU roctxRangePushA\b", out) and re.search(r"\bU roctxRangePop\b", out)


def _create(L, wl):
    from paper_1611_06721_amd import _lib as E
    grid = E.Grid((C.c_int32 * 3)(*wl.n), (C.c_double * 3)(*wl.length))
    cm = np.ascontiguousarray(wl.cell_mat, np.uint8)
    mats = (E.Material * max(1, len(wl.materials)))(
        *[E.Material(m.sigma, m.k1, m.k2, m.k3) for m in wl.materials])
    md = E.Materials(cm.ctypes.data_as(C.POINTER(C.c_uint8)), mats, len(wl.materials), wl.nu0)
    xs = np.ascontiguousarray(wl.edge_current, np.float64)
    src = E.Source(xs.ctypes.data_as(C.POINTER(C.c_double)), wl.waveform, wl.amp, wl.freq,
                   wl.tau, int(wl.ramp_steps))
    h = C.c_void_p()
    rc = L.ec_create(C.byref(grid), C.byref(md), C.byref(src), C.byref(h))
    return rc, h


@pytest.mark.parametrize("wl_fn", [lambda: synth.linear_c1(12), lambda: small_workload(),
                                   lambda: synth.nonlinear(48)])
def test_edge_counts_match_oracle(L, oracle_mod, wl_fn):
    wl = wl_fn()
    rc, h = _create(L, wl)
    assert rc == 0, L.ec_last_error(None)
    npad, nc, nn, ws = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
    assert L.ec_sizes(h, 8, C.byref(npad), C.byref(nc), C.byref(nn), C.byref(ws)) == 0
    O = oracle_mod.Problem(wl)
    assert npad.value == O.n_pad
    assert (nc.value, nn.value) == (int(O.C.sum()), int(O.N.sum()))
    assert ws.value > 13 * 8 * npad.value
    L.ec_destroy(h)


def test_rejects_divergent_source(L):
    wl = synth.linear_c1(12)
    xs = wl.edge_current.copy()
    xs[np.flatnonzero(xs)[0]] *= 1.5          # break Kirchhoff at two nodes
    wl.edge_current = xs
    rc, h = _create(L, wl)
    assert rc == -1 and not h.value
    assert b"divergence" in L.ec_last_error(None)


def test_rejects_source_on_conductor(L, oracle_mod):
    wl = small_workload()
    O = oracle_mod.Problem(wl)
    xs = wl.edge_current.copy()
    xs[np.flatnonzero(O.C)[0]] = 1.0
    wl.edge_current = xs
    rc, _ = _create(L, wl)
    assert rc == -1


@pytest.mark.parametrize("bad", ["grid", "sigma", "k3", "matid", "waveform"])
def test_rejects_bad_descriptors(L, bad):
    wl = small_workload()
    if bad == "grid":
        wl.n = (1, 6, 5)
    elif bad == "sigma":
        wl.materials = [synth.Material(0.0)]
    elif bad == "k3":
        wl.materials = [synth.Material(1e6, 0.0, 0.0, -1.0)]
    elif bad == "matid":
        cm = wl.cell_mat.copy()
        cm[0] = 7
        wl.cell_mat = cm
    elif bad == "waveform":
        wl.waveform = 9
    if bad == "grid":
        from paper_1611_06721_amd import _lib as E
        grid = E.Grid((C.c_int32 * 3)(1, 6, 5), (C.c_double * 3)(1, 1, 1))
        h = C.c_void_p()
        assert L.ec_create(C.byref(grid), None, None, C.byref(h)) == -1
        return
    rc, h = _create(L, wl)
    assert rc == -1 and not h.value


def test_sizes_window_cap_bounds(L):
    rc, h = _create(L, synth.linear_c1(12))
    assert rc == 0
    x = C.c_int64()
    assert L.ec_sizes(h, 0, None, None, None, C.byref(x)) == -1
    assert L.ec_sizes(h, 21, None, None, None, C.byref(x)) == -1
    a, b = C.c_int64(), C.c_int64()
    L.ec_sizes(h, 5, None, None, None, C.byref(a))
    L.ec_sizes(h, 10, None, None, None, C.byref(b))
    assert b.value > a.value
    assert L.ec_bind(h, None, None, 0, 5) == -1      # no workspace: rejected before any HIP call
    L.ec_destroy(h)
