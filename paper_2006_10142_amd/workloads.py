"""Seeded synthetic inputs for the implicit ADI wave solver.

This module only *draws* inputs: coefficient fields, initial states, source
time series and receiver positions.  It holds none of the scheme's arithmetic
(no stencil, no line solve, no time stepping), so the HIP library and the FP64
CPU oracle can both consume exactly the same arrays.

Conventions (the paper's grid, Sec. 2 eq. (f6), with N interior points per axis):
  * interior cell (i, j), 0-based, sits at x = (i+1) h, y = (j+1) h with
    h = 1/(N+1) on the unit square; walls are implicit zeros (eq. (CN3));
  * arrays are row-major ``a[j, i]`` (x fastest), shape ``(ny, nx)``;
  * ``c`` is a wave *speed*; the coefficient that multiplies the Laplacian in
    eq. (f1) is ``kappa = c**2``;
  * a point source of strength s(t) at one cell is the grid function
    f = s(t)/h**2 at that cell (a discrete delta), evaluated at t_n = n*dt,
    the level whose right-hand side it enters (eq. (CN1) uses f^k).

Inputs for an FP32 run are rounded to FP32 once, here; the oracle receives
those same values promoted to FP64, so a parity error measures solver error
only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "grid_h", "cell_centres", "smooth_field", "gaussian_pulse", "sine_mode",
    "ricker", "point_source_series", "Problem", "config_c1", "config_c2",
    "config_c3", "config_c3p", "config_c4", "config_c5", "batch_sizes",
]


def grid_h(n: int) -> float:
    """Grid step for n interior points on [0, 1]: h = 1/(n+1)."""
    return 1.0 / (n + 1)


def cell_centres(n: int) -> np.ndarray:
    """Interior node coordinates (i+1) h, i = 0..n-1, in FP64."""
    return (np.arange(n, dtype=np.float64) + 1.0) * grid_h(n)


def smooth_field(nx: int, ny: int, lo: float, hi: float, seed: int,
                 nbumps: int = 16) -> np.ndarray:
    """Seeded smooth random field on the interior grid, affinely mapped to [lo, hi].

    g(x, y) = sum_m a_m exp(-|x - x_m|^2 / (2 s_m^2)) with, from a PCG64 stream
    seeded by ``seed`` and drawn in this order: centres x_m ~ U[0,1]^2
    (nbumps x 2), widths s_m ~ U[0.05, 0.2], amplitudes a_m ~ U[-1, 1].
    The result is lo + (hi-lo) (g - min g)/(max g - min g) over the interior
    nodes, so its minimum is lo and its maximum is exactly hi.  FP64, (ny, nx).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.0, 1.0, size=(nbumps, 2))
    widths = rng.uniform(0.05, 0.2, size=nbumps)
    amps = rng.uniform(-1.0, 1.0, size=nbumps)
    x = (np.arange(nx, dtype=np.float64) + 1.0) / (nx + 1)
    y = (np.arange(ny, dtype=np.float64) + 1.0) / (ny + 1)
    g = np.zeros((ny, nx), dtype=np.float64)
    for (cx, cy), s, a in zip(centres, widths, amps):
        gx = np.exp(-((x - cx) ** 2) / (2.0 * s * s))
        gy = np.exp(-((y - cy) ** 2) / (2.0 * s * s))
        g += a * np.outer(gy, gx)
    gmin, gmax = float(g.min()), float(g.max())
    if gmax == gmin:
        return np.full((ny, nx), lo, dtype=np.float64)
    return lo + (hi - lo) * ((g - gmin) / (gmax - gmin))


def gaussian_pulse(nx: int, ny: int, sigma: float = 0.02,
                   centre=(0.5, 0.5)) -> np.ndarray:
    """u0 = exp(-((x-cx)^2 + (y-cy)^2) / (2 sigma^2)), amplitude 1, FP64 (ny, nx)."""
    x = (np.arange(nx, dtype=np.float64) + 1.0) / (nx + 1)
    y = (np.arange(ny, dtype=np.float64) + 1.0) / (ny + 1)
    gx = np.exp(-((x - centre[0]) ** 2) / (2.0 * sigma * sigma))
    gy = np.exp(-((y - centre[1]) ** 2) / (2.0 * sigma * sigma))
    return np.outer(gy, gx)


def sine_mode(nx: int, ny: int, kx: int = 1, ky: int = 1) -> np.ndarray:
    """sin(kx pi x) sin(ky pi y) on the interior nodes, FP64 (ny, nx)."""
    x = (np.arange(nx, dtype=np.float64) + 1.0) / (nx + 1)
    y = (np.arange(ny, dtype=np.float64) + 1.0) / (ny + 1)
    return np.outer(np.sin(ky * math.pi * y), np.sin(kx * math.pi * x))


def ricker(t, f0: float = 10.0, t0: Optional[float] = None):
    """Ricker wavelet s(t) = (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2), t0 = 1/f0."""
    if t0 is None:
        t0 = 1.0 / f0
    a = (math.pi * f0 * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def point_source_series(nsteps: int, dt: float, h: float, first_level: int,
                        f0: float = 10.0) -> np.ndarray:
    """Values of f at one source cell for nsteps consecutive steps.

    Step k of a run whose newest level is ``first_level`` builds its
    right-hand side on level n = first_level + k, so it uses
    f^n = ricker(n dt) / h^2.  FP64, shape (nsteps, 1).
    """
    n = first_level + np.arange(nsteps, dtype=np.float64)
    return (ricker(n * dt, f0) / (h * h)).reshape(nsteps, 1)


@dataclass
class Problem:
    """One synthetic run: grid, coefficient, initial levels, sources, receivers."""
    name: str
    nx: int
    ny: int
    h: float
    dt: float
    dtype: str                       # "f32" or "f64": the arithmetic type of the run
    nsteps: int
    c: Optional[np.ndarray] = None   # per-cell wave speed (ny, nx), already rounded to dtype
    c_scalar: float = 1.0            # used when c is None
    kappa: Optional[np.ndarray] = None  # per-cell kappa, when the run is posed in kappa
    u0: Optional[np.ndarray] = None  # level 0
    psi: Optional[np.ndarray] = None # du/dt at t=0 (None: zero)
    u_prev: Optional[np.ndarray] = None  # when the run starts from two given levels
    u_curr: Optional[np.ndarray] = None
    first_level: int = 1             # index n of u_curr
    src_idx: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    src_amp: Optional[np.ndarray] = None  # (nsteps, nsrc) values of f, dtype of the run
    rec_idx: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    start_mode: str = "ghost"        # how u^1 is made from u^0 and psi

    @property
    def np_dtype(self):
        return np.float32 if self.dtype == "f32" else np.float64

    def kappa_field(self) -> np.ndarray:
        """kappa = c^2 in FP64 from the (already rounded) inputs."""
        if self.kappa is not None:
            return np.asarray(self.kappa, dtype=np.float64)
        if self.c is None:
            return np.full((self.ny, self.nx), float(self.c_scalar) ** 2)
        c = np.asarray(self.c, dtype=np.float64)
        return c * c


def _round(a, dtype):
    return None if a is None else np.ascontiguousarray(np.asarray(a).astype(dtype))


def config_c1(dtype: str = "f64", nsteps: int = 200, n: int = 128,
              start_mode: str = "ghost") -> Problem:
    """Standing wave: N=n, h=1/(n+1), dt=h/2, kappa=1, u0=sin(pi x) sin(pi y), psi=0, f=0."""
    h = grid_h(n)
    dt_np = np.float32 if dtype == "f32" else np.float64
    return Problem("c1_standing_wave", n, n, h, 0.5 * h, dtype, nsteps,
                   c=None, c_scalar=1.0, u0=_round(sine_mode(n, n), dt_np),
                   start_mode=start_mode)


def config_c2(dtype: str = "f32", nsteps: int = 1000, n: int = 2048) -> Problem:
    """Gaussian pulse (sigma 0.02, centre (0.5, 0.5)), c=1, dt=h/2, zero walls, f=0."""
    h = grid_h(n)
    dt_np = np.float32 if dtype == "f32" else np.float64
    return Problem("c2_gaussian_pulse", n, n, h, 0.5 * h, dtype, nsteps,
                   c=None, c_scalar=1.0, u0=_round(gaussian_pulse(n, n), dt_np))


def config_c3(dtype: str = "f32", nsteps: int = 500, n: int = 8192,
              seed: int = 3) -> Problem:
    """Per-cell speed c in [1, 3] (16 Gaussian bumps, seed 3), dt = 0.4 h / max c,
    u^0 = u^1 = 0, Ricker (f0 = 10) at the centre cell (n/2, n/2) 1-based."""
    h = grid_h(n)
    dt_np = np.float32 if dtype == "f32" else np.float64
    c = _round(smooth_field(n, n, 1.0, 3.0, seed), dt_np)
    dt = 0.4 * h / float(np.max(c))
    zero = np.zeros((n, n), dtype=dt_np)
    ci = n // 2 - 1
    src_idx = np.array([ci * n + ci], dtype=np.int32)
    amp = _round(point_source_series(nsteps, dt, h, first_level=1), dt_np)
    return Problem("c3_heterogeneous_ricker", n, n, h, dt, dtype, nsteps, c=c,
                   u_prev=zero, u_curr=zero.copy(), first_level=1,
                   src_idx=src_idx, src_amp=amp)


def config_c3p(dtype: str = "f32", nsteps: int = 500, n: int = 8192,
               seed: int = 3) -> Problem:
    """The C3 speed field with a Gaussian u0 (sigma 0.02) instead of the source:
    a parity case whose solution is large everywhere the wave has travelled."""
    p = config_c3(dtype, nsteps, n, seed)
    p.name = "c3p_heterogeneous_pulse"
    p.u_prev = p.u_curr = None
    p.u0 = _round(gaussian_pulse(n, n), p.np_dtype)
    p.src_idx = np.zeros(0, np.int32)
    p.src_amp = None
    return p


def batch_sizes(count: int = 256, seed: int = 4) -> np.ndarray:
    """Square grid sizes N_s drawn uniformly from {256, 320, ..., 1024}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return 256 + 64 * rng.integers(0, 13, size=count)


def config_c4(dtype: str = "f32", nsteps: int = 500, count: int = 256,
              seed: int = 4) -> List[Problem]:
    """Batch of independent runs: N_s from batch_sizes, speed field seeded
    4000+s in [1, 3], Gaussian u0, dt_s = 0.4 h_s / max c_s, no sources."""
    dt_np = np.float32 if dtype == "f32" else np.float64
    out = []
    for s, n in enumerate(batch_sizes(count, seed)):
        n = int(n)
        h = grid_h(n)
        c = _round(smooth_field(n, n, 1.0, 3.0, 4000 + s), dt_np)
        dt = 0.4 * h / float(np.max(c))
        out.append(Problem(f"c4_sim{s}", n, n, h, dt, dtype, nsteps, c=c,
                           u0=_round(gaussian_pulse(n, n), dt_np)))
    return out


def config_c5(dtype: str = "f32", nsteps: int = 2000, n: int = 1024,
              seed: int = 5, target_seed: int = 6, nrec: int = 64):
    """Inverse-problem case: kappa in [1, 9] (seed 5), target kappa (seed 6),
    Ricker at the node nearest (0.5, 0.25), nrec receivers on the row nearest
    y = 0.1, dt = 0.4 h / 3, zero initial levels.

    Returns (problem, kappa_target).  The problem is posed in kappa directly.
    """
    h = grid_h(n)
    dt_np = np.float32 if dtype == "f32" else np.float64
    kappa = _round(smooth_field(n, n, 1.0, 9.0, seed), dt_np)
    kappa_t = _round(smooth_field(n, n, 1.0, 9.0, target_seed), dt_np)
    dt = 0.4 * h / 3.0
    # 1-based node nearest (0.5, 0.25): i = floor(0.5 (n+1) + 1/2), j = floor(0.25 (n+1) + 1/2)
    si = int(math.floor(0.5 * (n + 1) + 0.5)) - 1
    sj = int(math.floor(0.25 * (n + 1) + 0.5)) - 1
    rj = int(math.floor(0.1 * (n + 1) + 0.5)) - 1
    ri = [int(math.floor((r + 0.5) * (n + 1) / nrec + 0.5)) - 1 for r in range(nrec)]
    zero = np.zeros((n, n), dtype=dt_np)
    prob = Problem("c5_adjoint", n, n, h, dt, dtype, nsteps, kappa=kappa,
                   u_prev=zero, u_curr=zero.copy(), first_level=1,
                   src_idx=np.array([sj * n + si], dtype=np.int32),
                   src_amp=_round(point_source_series(nsteps, dt, h, 1), dt_np),
                   rec_idx=np.array([rj * n + i for i in ri], dtype=np.int32))
    return prob, kappa_t
