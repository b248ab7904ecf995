"""FP64 CPU oracle of the semi-explicit eddy-current scheme.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_1611_06721_amd``); the two meet only through the
seeded inputs of ``synth`` and the padded edge layout documented there.

Contents
--------
* ``ec_oracle.c`` (built to ``libecoracle.so``): FIT operators, plain CG,
  explicit Euler of eqs. (5a)-(7), power method for eq. (8), adjoint.
* ``startvec.py``: SPE (eq. 10, modified Gram-Schmidt) and POD (eqs. 11-14,
  SVD of the snapshot matrix) start vectors, written from Sec. III.
* ``adjoint.py``: the discrete adjoint of the explicit Euler loop (Joule
  loss, gradients with respect to sigma and k1).
* ``dense.py``: dense matrices of tiny grids for the pins (pseudo-inverse by
  eigendecomposition, Schur complement, closed-form decay).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecoracle.so")
SRC_PATH = os.path.join(HERE, "ec_oracle.c")

CLS_D, CLS_C, CLS_N = 0, 1, 2


def build(force=True):
    """Compile the C oracle with gcc (-O3, OpenMP)."""
    if not force and os.path.exists(LIB_PATH) and \
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    L = C.CDLL(LIB_PATH)
    L.or_create.restype = C.c_void_p
    L.or_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                            C.c_double, _u8, C.c_int, _dp, _dp, _dp, _dp, C.c_double]
    L.or_destroy.argtypes = [C.c_void_p]
    L.or_npad.restype = C.c_long
    L.or_npad.argtypes = [C.c_void_p]
    L.or_edge_class.argtypes = [C.c_void_p, _u8]
    L.or_msigma.argtypes = [C.c_void_p, _dp]
    L.or_cell_nu.argtypes = [C.c_void_p, _dp]
    L.or_apply.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.or_cell_B.argtypes = [C.c_void_p, _dp, _dp]
    L.or_curl.argtypes = [C.c_void_p, _dp, _dp]
    L.or_kn.argtypes = [C.c_void_p, _dp, _dp]
    L.or_kcnT.argtypes = [C.c_void_p, _dp, _dp]
    L.or_cg.restype = C.c_int
    L.or_cg.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int,
                        C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.or_waveform.restype = C.c_double
    L.or_waveform.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                              C.c_long, C.c_long, C.c_double]
    L.or_run.restype = C.c_int
    L.or_run.argtypes = [C.c_void_p, _dp, C.c_void_p, _dp, C.c_int, C.c_double,
                         C.c_double, C.c_double, C.c_long, C.c_double, C.c_long,
                         C.c_long, C.c_double, C.c_int, C.c_long, C.c_void_p,
                         C.c_void_p, C.c_void_p]
    L.or_power.restype = C.c_double
    L.or_power.argtypes = [C.c_void_p, _dp, C.c_int, C.c_double, C.c_uint]
    L.or_jn.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.or_jnT.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.or_dn_dk1.argtypes = [C.c_void_p, _dp, C.c_int, _dp]
    L.or_dmsig.argtypes = [C.c_void_p, C.c_int, _dp]
    L.or_set_threads.argtypes = [C.c_int]
    L.or_get_threads.restype = C.c_int
    _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Problem:
    """Oracle view of one workload (see synth.Workload)."""

    def __init__(self, wl):
        L = lib()
        self.wl = wl
        nx, ny, nz = wl.n
        lx, ly, lz = wl.length
        mats = wl.materials
        arr = lambda k: np.ascontiguousarray([getattr(m, k) for m in mats] or [0.0],
                                             dtype=np.float64)
        self._h = L.or_create(nx, ny, nz, lx, ly, lz,
                              np.ascontiguousarray(wl.cell_mat, dtype=np.uint8),
                              len(mats), arr("sigma"), arr("k1"), arr("k2"),
                              arr("k3"), wl.nu0)
        if not self._h:
            raise ValueError("oracle rejected the workload")
        self.n_pad = L.or_npad(self._h)
        self.cls = np.zeros(self.n_pad, np.uint8)
        L.or_edge_class(self._h, self.cls)
        self.msig = np.zeros(self.n_pad)
        L.or_msigma(self._h, self.msig)
        self.C = self.cls == CLS_C
        self.N = self.cls == CLS_N
        self.D = self.cls == CLS_D

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.or_destroy(h)
            except Exception:
                pass
            self._h = None

    # -- operators ---------------------------------------------------------
    def apply(self, x, state=None):
        """K x on non-Dirichlet edges, reluctivity taken from `state` (default x)."""
        x = np.ascontiguousarray(x, np.float64)
        v = x if state is None else np.ascontiguousarray(state, np.float64)
        y = np.zeros(self.n_pad)
        lib().or_apply(self._h, v, x, y)
        return y

    def kn(self, x):
        y = np.zeros(self.n_pad)
        lib().or_kn(self._h, np.ascontiguousarray(x, np.float64), y)
        return y

    def kcnT(self, a):
        y = np.zeros(self.n_pad)
        lib().or_kcnT(self._h, np.ascontiguousarray(a, np.float64), y)
        return y

    def curl(self, a):
        b = np.zeros(self.n_pad)
        lib().or_curl(self._h, np.ascontiguousarray(a, np.float64), b)
        return b

    def cell_B(self, a):
        nx, ny, nz = self.wl.n
        B = np.zeros(3 * nx * ny * nz)
        lib().or_cell_B(self._h, np.ascontiguousarray(a, np.float64), B)
        return B.reshape(-1, 3)

    def cell_nu(self, state):
        """Per-cell reluctivity evaluated at `state`."""
        self.apply(np.zeros(self.n_pad), state)
        nx, ny, nz = self.wl.n
        nu = np.zeros(nx * ny * nz)
        lib().or_cell_nu(self._h, nu)
        return nu

    # -- solver ------------------------------------------------------------
    def cg(self, b, x0=None, rtol=1e-10, maxit=100000):
        x = np.zeros(self.n_pad) if x0 is None else np.array(x0, np.float64)
        it, rel = C.c_int(0), C.c_double(0.0)
        st = lib().or_cg(self._h, np.ascontiguousarray(b, np.float64), x, rtol,
                         maxit, C.byref(it), C.byref(rel))
        return x, it.value, rel.value, st

    def source(self, m, dt):
        wl = self.wl
        i = lib().or_waveform(wl.waveform, wl.amp, wl.freq, wl.tau,
                              wl.ramp_steps, m, dt)
        b = i * wl.edge_current
        b[~self.N] = 0.0
        return b

    def run(self, dt, nsteps, rtol=1e-10, maxit=100000, A=None, sc=None, m0=0,
            rec_every=0):
        """Explicit Euler steps m0+1..m0+nsteps; returns (A, sc, rec, it_src, it_cpl)."""
        wl = self.wl
        A = np.zeros(self.n_pad) if A is None else np.array(A, np.float64)
        sc = np.zeros(self.n_pad) if sc is None else np.array(sc, np.float64)
        nrec = nsteps // rec_every if rec_every > 0 else 0
        rec = np.zeros((max(nrec, 1), self.n_pad))
        its = np.zeros(max(nsteps, 1), np.int32)
        itc = np.zeros(max(nsteps, 1), np.int32)
        st = lib().or_run(self._h, A, _ptr(sc),
                          np.ascontiguousarray(wl.edge_current, np.float64),
                          wl.waveform, wl.amp, wl.freq, wl.tau, wl.ramp_steps,
                          dt, m0, nsteps, rtol, maxit, rec_every,
                          _ptr(rec) if nrec else None, _ptr(its), _ptr(itc))
        if st:
            raise RuntimeError(f"oracle run failed with status {st}")
        return A, sc, rec[:nrec], its[:nsteps], itc[:nsteps]

    def power(self, A=None, iters=60, rtol=1e-12, seed=1):
        A = np.zeros(self.n_pad) if A is None else np.ascontiguousarray(A, np.float64)
        return lib().or_power(self._h, A, iters, rtol, seed)

    # -- adjoint pieces ------------------------------------------------------
    def n_c(self, a):
        """N(a) = [K(nu(a)) a]_C for a restricted to C (the conducting block)."""
        ac = np.where(self.C, a, 0.0)
        return np.where(self.C, self.apply(ac, ac), 0.0)

    def jn(self, a, v):
        y = np.zeros(self.n_pad)
        lib().or_jn(self._h, np.ascontiguousarray(a, np.float64),
                    np.ascontiguousarray(v, np.float64), y)
        return y

    def jnT(self, a, lam):
        y = np.zeros(self.n_pad)
        lib().or_jnT(self._h, np.ascontiguousarray(a, np.float64),
                     np.ascontiguousarray(lam, np.float64), y)
        return y

    def dn_dk1(self, a, mat=1):
        y = np.zeros(self.n_pad)
        lib().or_dn_dk1(self._h, np.ascontiguousarray(a, np.float64), int(mat), y)
        return y

    def dmsig(self, mat=1):
        y = np.zeros(self.n_pad)
        lib().or_dmsig(self._h, int(mat), y)
        return y

    def schur(self, w, rtol=1e-12):
        """S w = K_cn K_n^+ K_cn^T w on C edges (w read on C)."""
        s, _, _, st = self.cg(self.kcnT(np.where(self.C, w, 0.0)), rtol=rtol)
        if st:
            raise RuntimeError(f"oracle CG failed with status {st}")
        return np.where(self.C, self.apply(np.where(self.N, s, 0.0), np.zeros(self.n_pad)), 0.0)


def set_threads(n):
    lib().or_set_threads(int(n))


def get_threads():
    return lib().or_get_threads()
