"""Seeded synthetic workloads shared by the CPU oracle and the HIP library.

This module holds geometry and input data only: grid sizes, the per-cell
material map, the coil's edge currents and the seeded random draws.  It holds
none of the method's arithmetic (no curl, no reluctivity, no solver), so the
oracle and the GPU path can both take their inputs from here without sharing
any computation.

Edge-array layout (the interface both sides agree on)
-----------------------------------------------------
Edge unknowns live in one "padded" float array of length ``3 * S`` with
``S = (nx+1)*(ny+1)*(nz+1)``.  Block ``c`` (0 = x, 1 = y, 2 = z) holds the
edges of direction ``c``; inside a block the edge anchored at node (i, j, k)
sits at ``(k*(ny+1) + j)*(nx+1) + i`` (i fastest).  The x-edge at (i, j, k)
joins node (i, j, k) to (i+1, j, k); y and z edges likewise.  Slots with
i = nx (x block), j = ny (y block) or k = nz (z block) are padding and stay
zero.  Cells are indexed ``(k*ny + j)*nx + i``.

Workloads (sizes of the paper's TEAM-10 runs, Sec. IV; the benchmark geometry
itself is not reproduced: a cube stands in for it)
----------------------------------------------------------------------------
* conductor: cells whose centres lie in [1/3, 2/3]^3 of the unit cube;
* coil: closed square edge loops around the z axis, weighted so that the coil
  is a band [N/12, N/4] from the wall (2 cells thick at N = 12) and
  [5N/12, 7N/12] in z, carrying a uniform current density J0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MU0 = 4.0e-7 * math.pi
NU0 = 1.0 / MU0

# waveform ids (identical numbering on both sides of the C-ABI)
WF_DC, WF_SIN, WF_RAMP, WF_EXP = 0, 1, 2, 3

# Brauer reluctivity coefficients of the nonlinear workloads
BRAUER = (3.8, 2.17, 396.2)


@dataclass
class Material:
    sigma: float
    k1: float = 0.0
    k2: float = 0.0
    k3: float = NU0


@dataclass
class Workload:
    """A complete problem description: grid, materials, coil and waveform."""
    name: str
    n: tuple            # cells per axis (nx, ny, nz)
    length: tuple       # box side lengths [m]
    cell_mat: np.ndarray    # uint8, nx*ny*nz, 0 = nonconducting (nu0)
    materials: list         # Material for ids 1..len
    edge_current: np.ndarray  # float64 padded edge array, A per unit i_S
    waveform: int = WF_SIN
    amp: float = 1.0
    freq: float = 50.0
    tau: float = 0.5
    ramp_steps: int = 1
    nu0: float = NU0
    extra: dict = field(default_factory=dict)

    @property
    def h(self):
        return tuple(l / c for l, c in zip(self.length, self.n))

    @property
    def S(self):
        nx, ny, nz = self.n
        return (nx + 1) * (ny + 1) * (nz + 1)

    @property
    def n_pad(self):
        return 3 * self.S


def edge_slot(n, comp, i, j, k):
    """Position of edge (comp, i, j, k) in the padded array (see module doc)."""
    nx, ny, nz = n
    S = (nx + 1) * (ny + 1) * (nz + 1)
    return comp * S + (k * (ny + 1) + j) * (nx + 1) + i


def conductor_range(N):
    """Cell indices i with centre (i + 1/2)/N inside [1/3, 2/3] (integer test)."""
    lo = None
    hi = None
    for i in range(N):
        c6 = 6 * i + 3           # 6*(i+1/2)
        if 2 * N <= c6 <= 4 * N:
            lo = i if lo is None else lo
            hi = i
    return lo, hi


def box_cell_mat(n, lo, hi, mat_id=1):
    """uint8 cell map with material `mat_id` on cells lo..hi (inclusive) per axis."""
    nx, ny, nz = n
    cm = np.zeros((nz, ny, nx), dtype=np.uint8)
    cm[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = mat_id
    return cm.reshape(-1)


def _overlap(a0, a1, b0, b1):
    return max(0.0, min(a1, b1) - max(a0, b0))


def square_loop(n, arr, d, k, current):
    """Add a closed square loop of x/y edges at z-node k, corners (d,d)-(N-d,N-d).

    Counter-clockwise seen from +z.  Every node has as much current leaving as
    entering, so the loop is discretely divergence free.
    """
    nx, ny, _ = n
    for i in range(d, nx - d):
        arr[edge_slot(n, 0, i, d, k)] += current
        arr[edge_slot(n, 0, i, ny - d, k)] -= current
    for j in range(d, ny - d):
        arr[edge_slot(n, 1, nx - d, j, k)] += current
        arr[edge_slot(n, 1, d, j, k)] -= current


def coil_current(N, J0, length=1.0):
    """Edge currents of the band coil on an N^3 cube grid (A per unit i_S)."""
    n = (N, N, N)
    h = length / N
    arr = np.zeros(3 * (N + 1) ** 3, dtype=np.float64)
    r0, r1 = N / 12.0, N / 4.0
    z0, z1 = 5.0 * N / 12.0, 7.0 * N / 12.0
    for d in range(1, N // 2):
        wd = _overlap(d - 0.5, d + 0.5, r0, r1)
        if wd <= 0.0:
            continue
        for k in range(1, N):
            wk = _overlap(k - 0.5, k + 0.5, z0, z1)
            if wk <= 0.0:
                continue
            square_loop(n, arr, d, k, J0 * h * h * wd * wk)
    return arr


def cube_workload(name, N, material, J0, waveform, **wf):
    lo, hi = conductor_range(N)
    n = (N, N, N)
    cm = box_cell_mat(n, (lo,) * 3, (hi,) * 3)
    return Workload(name=name, n=n, length=(1.0, 1.0, 1.0), cell_mat=cm,
                    materials=[material], edge_current=coil_current(N, J0),
                    waveform=waveform, extra={"conductor": (lo, hi), "J0": J0},
                    **wf)


# Amplitude of the nonlinear workloads.  The ramped 1e6 A/m^2 of the plain
# case leaves |B| in the iron far below the knee of the Brauer curve, so the
# nonlinear runs use a current density that drives the iron surface cells
# into saturation (peak |B| of about 1.5 T, found with an oracle run at N = 24).
J0_NONLINEAR = 3.0e6


def linear_c1(N=12):
    """12^3 cells, 4^3 linear conductor sigma = 1e6, 50 Hz sine coil, 1e6 A/m^2."""
    return cube_workload("linear", N, Material(1.0e6, 0.0, 0.0, NU0), 1.0e6,
                         WF_SIN, freq=50.0)


def nonlinear(N=48, ramp_steps=1000, J0=None, sigma=2.0e6, brauer=BRAUER, name=None):
    """N^3 cells, Brauer iron conductor, coil current ramped linearly."""
    k1, k2, k3 = brauer
    return cube_workload(name or f"nonlinear{N}", N, Material(sigma, k1, k2, k3),
                         J0_NONLINEAR if J0 is None else J0, WF_RAMP,
                         ramp_steps=ramp_steps)


def batch_draws(count=64, seed=161106721):
    """Per-instance (N, sigma, k1, k2, k3) of the uneven batch workload."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        N = int(rng.integers(16, 65))
        sigma = 10.0 ** rng.uniform(5.0, 7.0)
        ks = [b * (1.0 + rng.uniform(-0.1, 0.1)) for b in BRAUER]
        out.append((N, sigma, *ks))
    return out


def batch_workloads(count=64, seed=161106721, ramp_steps=1000):
    return [nonlinear(N, ramp_steps=ramp_steps, sigma=s, brauer=(a, b, c),
                      name=f"batch{idx}_N{N}")
            for idx, (N, s, a, b, c) in enumerate(batch_draws(count, seed))]


def random_vector(n_pad, mask, seed):
    """Seeded standard-normal vector, zero where `mask` is False."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n_pad)
    v[~mask] = 0.0
    return v
