"""torch-facing wrapper of the C-ABI: device memory and streams come from torch,
every operation runs in the library's HIP kernels."""
from __future__ import annotations

import contextlib
import ctypes as C
import sys

import numpy as np
import torch

from . import _lib as L

INFO_BYTES = C.sizeof(L.SolveInfo)
_INFO_DTYPE = np.dtype([("iters", "<i4"), ("outer_iters", "<i4"), ("status", "<i4"),
                        ("basis_cols", "<i4"), ("rel_res", "<f8"), ("b_norm", "<f8"),
                        ("pod_info", "<f8"), ("r0_rel", "<f8")])
assert _INFO_DTYPE.itemsize == INFO_BYTES


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def solve_opts(rtol=1e-8, maxit=100000, precision=L.PREC_FP64, inner_rtol=1e-5,
               inner_maxit=200, outer_max=8):
    return L.SolveOpts(rtol, maxit, precision, inner_rtol, inner_maxit, outer_max)


def step_opts(method=L.SV_SPE, window=8, pod_kmax=None, pod_eps=1e-4, graph_iters=(0, 0),
              graph_serial=False, **solve):
    """graph_iters: PCG iterations budgeted per solve (source, coupling) in a
    captured step; 0 = maxit.  graph_serial: capture the step as one chain
    (no branch for the history pushes)."""
    kmax = window if pod_kmax is None else pod_kmax
    return L.StepOpts(method, window, kmax, pod_eps, solve_opts(**solve),
                      (C.c_int32 * 2)(*graph_iters), 1 if graph_serial else 0)


def info_array(info_tensor):
    """Device info records -> numpy structured array (synchronises)."""
    raw = info_tensor.detach().cpu().numpy().view(np.uint8)
    return raw.view(_INFO_DTYPE)


class Problem:
    """One FIT eddy-current problem bound to a torch device and stream.

    `wl` is any object with the fields of synth.Workload (n, length, cell_mat,
    materials, edge_current, waveform, amp, freq, tau, ramp_steps, nu0).

    The library runs on its own (capturable, non-default) torch stream; every
    call first waits for the caller's current stream and makes the caller's
    stream wait for the library's work, so tensors can be used as usual."""

    def __init__(self, wl, window_cap=8, device="cuda:0", stream=None):
        self.lib = L.load()
        self.device = torch.device(device)
        grid = L.Grid((C.c_int32 * 3)(*wl.n), (C.c_double * 3)(*wl.length))
        self._cell = np.ascontiguousarray(wl.cell_mat, dtype=np.uint8)
        mats = (L.Material * max(1, len(wl.materials)))(
            *[L.Material(m.sigma, m.k1, m.k2, m.k3) for m in wl.materials])
        mdesc = L.Materials(self._cell.ctypes.data_as(C.POINTER(C.c_uint8)), mats,
                            len(wl.materials), wl.nu0)
        self._xs = np.ascontiguousarray(wl.edge_current, dtype=np.float64)
        src = L.Source(self._xs.ctypes.data_as(C.POINTER(C.c_double)), wl.waveform, wl.amp,
                       wl.freq, wl.tau, int(wl.ramp_steps))
        h = C.c_void_p()
        L.check(self.lib.ec_create(C.byref(grid), C.byref(mdesc), C.byref(src), C.byref(h)))
        self.h = h
        npad, nc, nn, ws = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        self._chk(self.lib.ec_sizes(self.h, window_cap, C.byref(npad), C.byref(nc),
                                    C.byref(nn), C.byref(ws)))
        self.n_pad, self.n_c, self.n_n = npad.value, nc.value, nn.value
        self.window_cap = window_cap
        self.workspace = torch.empty(ws.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        with self._on_stream():
            self._chk(self.lib.ec_bind(self.h, C.c_void_p(self.stream.cuda_stream),
                                       C.c_void_p(self._ws_ptr), ws.value, window_cap))
        self.wl = wl

    # ------------------------------------------------------------ helpers
    def _chk(self, code):
        return L.check(code, self.h)

    @contextlib.contextmanager
    def _on_stream(self):
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)
        try:
            yield
        finally:
            if cur.cuda_stream != self.stream.cuda_stream:
                cur.wait_stream(self.stream)

    def close(self):
        """Destroy the handle after the library's stream has drained (the
        workspace tensor is released with this object).  Graphs and batches
        that use the problem must be closed first."""
        h = getattr(self, "h", None)
        if h is not None and getattr(self, "lib", None) is not None:
            self.stream.synchronize()
            self.lib.ec_destroy(h)
        self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the HIP runtime (or a profiler wrapped around
        # it) may already be gone: leave the process teardown to free it
        if not _finalizing():
            self.close()

    def zeros(self):
        return torch.zeros(self.n_pad, dtype=torch.float64, device=self.device)

    def tensor(self, a):
        return torch.as_tensor(np.ascontiguousarray(a, np.float64), device=self.device)

    def info(self, n=1):
        return torch.zeros(n * INFO_BYTES, dtype=torch.uint8, device=self.device)

    # ------------------------------------------------------------ calls
    def apply(self, op, x, out=None):
        y = self.zeros() if out is None else out
        with self._on_stream():
            self._chk(self.lib.ec_apply(self.h, op, _ptr(x), _ptr(y)))
        return y

    def solve(self, b, x=None, seq=L.SEQ_USER, method=L.SV_ZERO, window=1, info=None, **opts):
        x = self.zeros() if x is None else x
        o = solve_opts(**opts)
        with self._on_stream():
            self._chk(self.lib.ec_solve(self.h, seq, method, window, _ptr(b), _ptr(x),
                                        C.byref(o), _ptr(info)))
        return x

    def solve_static(self, b, x=None, method=L.SV_ZERO, info=None, **opts):
        """ec_solve_static: the FP64 PCG of solve() with its scratch in the
        library's static device array (ZERO or PREV start)."""
        x = self.zeros() if x is None else x
        o = solve_opts(**opts)
        with self._on_stream():
            self._chk(self.lib.ec_solve_static(self.h, method, _ptr(b), _ptr(x), C.byref(o),
                                               _ptr(info)))
        return x

    def set_gauge_penalty(self, factor):
        with self._on_stream():
            self._chk(self.lib.ec_set_gauge_penalty(self.h, factor))

    def set_pcg_kernel(self, kind):
        """0 node-parallel, 1 2.5D (LDS-staged), -1 default for the grid size."""
        self._chk(self.lib.ec_set_pcg_kernel(self.h, int(kind)))

    def tune_pcg(self, cache_path=None):
        """(column width or 0, planes per block, us per iteration) of the
        fastest PCG iteration kernel for this grid (applied to the handle)."""
        ti, kb, us = C.c_int32(), C.c_int32(), C.c_double()
        with self._on_stream():
            self._chk(self.lib.ec_tune_pcg(self.h, cache_path.encode() if cache_path else None,
                                           C.byref(ti), C.byref(kb), C.byref(us)))
        return ti.value, kb.value, us.value

    def set_dependency_tol(self, tol):
        with self._on_stream():
            self._chk(self.lib.ec_set_dependency_tol(self.h, tol))

    def history_reset(self, seq):
        with self._on_stream():
            self._chk(self.lib.ec_history_reset(self.h, seq))

    def history_push(self, seq, method, window, x):
        with self._on_stream():
            self._chk(self.lib.ec_history_push(self.h, seq, method, window, _ptr(x)))

    def start_vector(self, seq, method, window, b, pod_kmax=None, pod_eps=1e-4, x0=None,
                     info=None):
        x0 = self.zeros() if x0 is None else x0
        kmax = window if pod_kmax is None else pod_kmax
        with self._on_stream():
            self._chk(self.lib.ec_start_vector(self.h, seq, method, window, kmax, pod_eps,
                                               _ptr(b), _ptr(x0), _ptr(info)))
        return x0

    def set_state(self, A, **opts):
        o = solve_opts(**opts)
        with self._on_stream():
            self._chk(self.lib.ec_set_state(self.h, _ptr(A), C.byref(o)))

    def step(self, A, m, dt, opts, info=None):
        with self._on_stream():
            self._chk(self.lib.ec_step(self.h, m, dt, _ptr(A), C.byref(opts), _ptr(info)))

    def run(self, A, m0, nsteps, dt, opts, info=None):
        with self._on_stream():
            self._chk(self.lib.ec_run(self.h, m0, nsteps, dt, _ptr(A), C.byref(opts),
                                      _ptr(info)))

    def counters(self):
        v = [C.c_int64() for _ in range(4)]
        w = C.c_int32()
        with self._on_stream():
            self._chk(self.lib.ec_counters(self.h, *[C.byref(x) for x in v], C.byref(w)))
        return {"steps": v[0].value, "iters_src": v[1].value, "iters_cpl": v[2].value,
                "iters_adj": v[3].value, "worst_status": w.value}

    def counters_reset(self):
        with self._on_stream():
            self._chk(self.lib.ec_counters_reset(self.h))

    def set_step(self, m):
        with self._on_stream():
            self._chk(self.lib.ec_set_step(self.h, m))

    def cfl(self, A=None, iters=60, rtol=1e-12):
        A = self.zeros() if A is None else A
        lam = C.c_double()
        with self._on_stream():
            self._chk(self.lib.ec_cfl(self.h, _ptr(A), iters, rtol, C.byref(lam)))
        return lam.value

    def cfl_estimate(self, A=None, iters=30, rtol=1e-10, method=L.SV_SPE, window=8,
                     jacobian=True, lam=None, rec=None):
        """Device power-method estimate of |lambda|_max (eq. 8) at state A into
        the device scalar `lam` (a new float64 tensor if None), asynchronously."""
        A = self.zeros() if A is None else A
        lam = torch.zeros(1, dtype=torch.float64, device=self.device) if lam is None else lam
        with self._on_stream():
            self._chk(self.lib.ec_cfl_estimate(self.h, _ptr(A), int(iters), float(rtol),
                                               int(method), int(window), 1 if jacobian else 0,
                                               _ptr(lam), _ptr(rec)))
        return lam

    def set_adaptive_dt(self, lam, safety=0.5):
        """Steps read the device estimate `lam` and halve dt to meet it (None:
        fixed steps).  The tensor must outlive the steps that use it."""
        self._adapt_lam = lam
        with self._on_stream():
            self._chk(self.lib.ec_set_adaptive_dt(self.h, _ptr(lam), float(safety)))

    def clock(self):
        m, t, dt = C.c_int64(), C.c_double(), C.c_double()
        with self._on_stream():
            self._chk(self.lib.ec_clock(self.h, C.byref(m), C.byref(t), C.byref(dt)))
        return m.value, t.value, dt.value

    def implicit_step(self, A, m, dt, newton_rtol=1e-10, max_newton=20, gmres_m=20,
                      gmres_max=400, gmres_rtol=1e-8, inner_rtol=1e-10, method=L.SV_SPE,
                      window=8):
        """One implicit Euler step with Newton-GMRES (ec_implicit_step);
        returns the step's counts and residual norms."""
        o = L.ImplicitOpts(float(newton_rtol), int(max_newton), int(gmres_m), int(gmres_max),
                           float(gmres_rtol), float(inner_rtol), int(method), int(window))
        inf = L.ImplicitInfo()
        with self._on_stream():
            self._chk(self.lib.ec_implicit_step(self.h, int(m), float(dt), _ptr(A), C.byref(o),
                                                C.byref(inf)))
        return {"newton_iters": inf.newton_iters, "gmres_iters": inf.gmres_iters,
                "kn_solves": inf.kn_solves, "status": inf.status, "res0": inf.res0,
                "res": inf.res}

    def set_mass(self, kind, method=L.SV_SPE, window=8, rtol=1e-10, maxit=200):
        """Conductivity matrix of the step: MASS_LUMPED (diagonal FIT) or
        MASS_CONSISTENT (edge-element mass, M_c y = g solved every step)."""
        with self._on_stream():
            self._chk(self.lib.ec_set_mass(self.h, int(kind), int(method), int(window),
                                           float(rtol), int(maxit)))

    def mass_apply(self, x, out=None):
        y = self.zeros() if out is None else out
        with self._on_stream():
            self._chk(self.lib.ec_mass_apply(self.h, _ptr(x), _ptr(y)))
        return y

    def mass_solve(self, g, out=None, info=None):
        y = self.zeros() if out is None else out
        with self._on_stream():
            self._chk(self.lib.ec_mass_solve(self.h, _ptr(g), _ptr(y), _ptr(info)))
        return y

    def mass_counters(self):
        a, b = C.c_int64(), C.c_int64()
        with self._on_stream():
            self._chk(self.lib.ec_mass_counters(self.h, C.byref(a), C.byref(b)))
        return {"solves": a.value, "iters": b.value}

    def set_material(self, mat_id, sigma, k1, k2, k3):
        m = L.Material(float(sigma), float(k1), float(k2), float(k3))
        with self._on_stream():
            self._chk(self.lib.ec_set_material(self.h, int(mat_id), C.byref(m)))

    def adjoint_workspace(self, n_steps, every):
        b = C.c_int64()
        self._chk(self.lib.ec_adjoint_sizes(self.h, int(n_steps), int(every), C.byref(b)))
        ws = torch.empty(b.value + 256, dtype=torch.uint8, device=self.device)
        return ws, (-ws.data_ptr()) % 256, b.value

    def adjoint_forward(self, A, n_steps, dt, every, opts, ws):
        """Joule loss of n_steps steps from A (device scalar); A ends at a^M."""
        buf, off, nb = ws
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        with self._on_stream():
            self._chk(self.lib.ec_adjoint_forward(self.h, int(n_steps), float(dt), int(every),
                                                  C.byref(opts), C.c_void_p(buf.data_ptr() + off),
                                                  nb, _ptr(A), _ptr(loss)))
        return loss

    def adjoint_backward(self, n_steps, dt, every, opts, ws, mat_id=1):
        """(dL/dsigma, dL/dk1) of material mat_id as a device tensor [2]."""
        buf, off, nb = ws
        g = torch.zeros(2, dtype=torch.float64, device=self.device)
        with self._on_stream():
            self._chk(self.lib.ec_adjoint_backward(self.h, int(n_steps), float(dt), int(every),
                                                   C.byref(opts),
                                                   C.c_void_p(buf.data_ptr() + off), nb,
                                                   int(mat_id), _ptr(g)))
        return g

    def graph_capture(self, A, dt, opts, info=None):
        g = C.c_void_p()
        with self._on_stream():
            self._chk(self.lib.ec_graph_capture_step(self.h, dt, _ptr(A), C.byref(opts),
                                                     _ptr(info), C.byref(g)))
        return Graph(self, g)


class Graph:
    """A captured step; launch() replays it on the problem's stream."""

    def __init__(self, prob, g):
        self.prob, self.lib, self.g = prob, prob.lib, g

    def launch(self):
        with self.prob._on_stream():
            L.check(self.lib.ec_graph_launch(self.g, C.c_void_p(self.prob.stream.cuda_stream)))

    def launch_raw(self):
        """Replay without stream hand-offs (the caller synchronises)."""
        L.check(self.lib.ec_graph_launch(self.g, C.c_void_p(self.prob.stream.cuda_stream)))

    def close(self):
        if getattr(self, "g", None):
            self.prob.stream.synchronize()
            self.lib.ec_graph_destroy(self.g)
        self.g = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if not _finalizing():
            self.close()


class Batch:
    """Problems of uneven size stepped together: every kernel of a step (PCG
    iterations, start vectors, history pushes, the conducting update) is one
    launch for all problems.  All problems must share one stream: create them
    with Problem(wl, stream=s) for a common torch stream s."""

    def __init__(self, problems):
        self.problems = list(problems)
        p0 = self.problems[0]
        self.lib, self.device, self.stream = p0.lib, p0.device, p0.stream
        if any(p.stream.cuda_stream != p0.stream.cuda_stream for p in self.problems):
            raise ValueError("all problems of a batch must share one stream")
        n = len(self.problems)
        self._hs = (C.c_void_p * n)(*[p.h.value for p in self.problems])
        b = C.c_int64()
        L.check(self.lib.ec_batch_sizes(n, self._hs, C.byref(b)))
        self.workspace = torch.empty(b.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        out = C.c_void_p()
        with p0._on_stream():
            L.check(self.lib.ec_batch_create(n, self._hs,
                                             C.c_void_p(self.workspace.data_ptr() + off),
                                             b.value, C.byref(out)))
        self.b = out

    def _args(self, dt, A):
        n = len(self.problems)
        dts = (C.c_double * n)(*[float(d) for d in dt])
        ptrs = (C.c_void_p * n)(*[a.data_ptr() for a in A])
        return dts, ptrs

    def step(self, dt, A, opts, m=-1):
        dts, ptrs = self._args(dt, A)
        with self.problems[0]._on_stream():
            L.check(self.lib.ec_batch_step(self.b, int(m), dts, ptrs, C.byref(opts)))

    def run(self, m0, nsteps, dt, A, opts):
        dts, ptrs = self._args(dt, A)
        with self.problems[0]._on_stream():
            L.check(self.lib.ec_batch_run(self.b, int(m0), int(nsteps), dts, ptrs, C.byref(opts)))

    def graph_capture(self, dt, A, opts):
        dts, ptrs = self._args(dt, A)
        g = C.c_void_p()
        with self.problems[0]._on_stream():
            L.check(self.lib.ec_batch_graph_capture(self.b, dts, ptrs, C.byref(opts),
                                                    C.byref(g)))
        return Graph(self.problems[0], g)

    def set_tiles(self, tiles_per_block):
        L.check(self.lib.ec_batch_set_tiles(self.b, int(tiles_per_block)))

    def autotune(self, cache_path=None):
        f, us = C.c_int32(), C.c_double()
        with self.problems[0]._on_stream():
            L.check(self.lib.ec_batch_autotune(self.b, cache_path.encode() if cache_path else None,
                                               C.byref(f), C.byref(us)))
        return f.value, us.value

    def close(self):
        if getattr(self, "b", None):
            self.stream.synchronize()
            self.lib.ec_batch_destroy(self.b)
        self.b = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if not _finalizing():
            self.close()

