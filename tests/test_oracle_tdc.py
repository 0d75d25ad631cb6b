"""Pins of the oracle's step for eq. (CN1) with a time-dependent coefficient
(kappa at t_{k+1} on the Laplacian of u^{k+1}, kappa at t_{k-1} on that of u^{k-1}):

  * the unfactored eq. (CN1) with c^{k+1}, c^{k-1}, as printed, solved densely for
    u^{k+1}: the ADI step differs from it by a term of order dt^6 (a wrong or
    missing coefficient term leaves an O(dt^3) or O(dt^5) gap);
  * second-order convergence to a manufactured solution of u_tt = kappa(t,x,y) Lap u + f;
  * the discrete closed form of a grid mode under a spatially constant kappa(t);
  * for a coefficient constant in time it is the plain step."""
import math

import numpy as np
import pytest

from tests.conftest import rel_l2
from tests.test_oracle_pins import dense_ops


def grid(nx, ny, h):
    x = (np.arange(nx) + 1) * h
    y = (np.arange(ny) + 1) * h
    return np.meshgrid(x, y)        # (ny, nx) arrays


def test_constant_coefficient_is_the_plain_step(oracle_lib):
    rng = np.random.default_rng(1)
    nx, ny, h, dt = 12, 9, 0.1, 0.03
    kap = rng.uniform(1.0, 3.0, (ny, nx))
    up, uc, f = (rng.standard_normal((ny, nx)) for _ in range(3))
    got = oracle_lib.step_tdc(kap, kap, up, uc, h, dt, f=f)
    ref = oracle_lib.step_parts(kap, up, uc, h, dt, f=f)["u_next"]
    assert rel_l2(got, ref) <= 1e-13


def _cn1_tdc_dense(kp, kn, up, uc, f, h, dt):
    """eq. (CN1) as printed: (u+ - 2u + u-)/dt^2 - kn/2 Lap u+ - kp/2 Lap u- = f, for u+."""
    ny, nx = uc.shape
    Lx, Ly = dense_ops(nx, ny, h)
    L = Lx + Ly
    n = nx * ny
    Kn, Kp = np.diag(kn.ravel()), np.diag(kp.ravel())
    A = np.eye(n) / dt ** 2 - 0.5 * Kn @ L
    rhs = (2 * uc.ravel() - up.ravel()) / dt ** 2 + 0.5 * Kp @ L @ up.ravel() + f.ravel()
    return np.linalg.solve(A, rhs).reshape(ny, nx)


def test_step_vs_unfactored_cn1_gap_is_order_dt6(oracle_lib):
    nx, ny = 9, 8
    h = 1.0 / 10.0
    rng = np.random.default_rng(7)
    ka = rng.uniform(1.0, 2.0, (ny, nx))
    kb = rng.uniform(-1.0, 1.0, (ny, nx))        # d kappa / dt
    X, Y = grid(nx, ny, h)
    base = np.sin(math.pi * X) * np.sin(math.pi * Y) + 0.3 * np.sin(3 * math.pi * X) * np.sin(2 * math.pi * Y)
    f = 0.7 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    t = 0.5
    gaps = []
    for dt in (0.04 * h, 0.02 * h, 0.01 * h):
        kp, kn = ka + (t - dt) * kb, ka + (t + dt) * kb
        up = base
        uc = base * math.cos(math.sqrt(2) * math.pi * dt)
        ref = _cn1_tdc_dense(kp, kn, up, uc, f, h, dt)
        got = oracle_lib.step_tdc(kp, kn, up, uc, h, dt, f=f)
        gaps.append(np.linalg.norm((got - ref).ravel()))
    orders = [math.log2(gaps[k] / gaps[k + 1]) for k in range(2)]
    for o in orders:
        assert 5.7 < o < 6.3, (gaps, orders)


def _manufactured_error(oracle_lib, n, T=0.25, w=2 * math.pi):
    h = 1.0 / (n + 1)
    dt = 0.5 * h
    X, Y = grid(n, n, h)
    phi = np.sin(math.pi * X) * np.sin(math.pi * Y)
    kappa = lambda t: 1.0 + 0.5 * math.sin(2.0 * t) * (1.0 + X * Y)
    exact = lambda t: math.cos(w * t) * phi
    # u_tt = kappa Lap u + f with Lap phi = -2 pi^2 phi
    force = lambda t: (-w * w + 2 * math.pi ** 2 * kappa(t)) * math.cos(w * t) * phi
    steps = int(round(T / dt))
    up, uc = exact(0.0), exact(dt)
    for k in range(1, steps):
        t = k * dt
        up, uc = uc, oracle_lib.step_tdc(kappa(t - dt), kappa(t + dt), up, uc, h, dt, f=force(t))
    return rel_l2(uc, exact(steps * dt))


def test_converges_to_manufactured_solution_at_second_order(oracle_lib):
    errs = [_manufactured_error(oracle_lib, n) for n in (15, 31, 63)]
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    for o in orders:
        assert 1.85 < o < 2.15, (errs, orders)


def test_mode_under_spatially_constant_kappa_of_t(oracle_lib):
    """u = a^k sin(pi x) sin(pi y): each 1-D second difference multiplies the mode by
    -lam, lam = 4 sin^2(pi h / 2) / h^2, so the step is a scalar recurrence."""
    n = 40
    h = 1.0 / (n + 1)
    dt = 0.6 * h
    X, Y = grid(n, n, h)
    phi = np.sin(math.pi * X) * np.sin(math.pi * Y)
    kap = lambda t: 1.0 + 0.5 * math.sin(3.0 * t)
    lam = 4.0 * math.sin(math.pi * h / 2.0) ** 2 / (h * h)
    beta = 0.5 * dt * dt
    a_prev, a_curr = 1.0, math.cos(math.sqrt(2) * math.pi * dt)
    up, uc = a_prev * phi, a_curr * phi
    for k in range(1, 120):
        t = k * dt
        kp, kn = kap(t - dt), kap(t + dt)
        up, uc = uc, oracle_lib.step_tdc(np.full_like(phi, kp), np.full_like(phi, kn), up, uc, h, dt)
        # (1 + beta kn lam)^2 d = beta (2 kn (-2 lam) a + (kp - kn) (-2 lam) a_prev)
        d = -2.0 * beta * lam * (2.0 * kn * a_curr + (kp - kn) * a_prev) / (1.0 + beta * kn * lam) ** 2
        a_prev, a_curr = a_curr, 2.0 * a_curr - a_prev + d
    assert rel_l2(uc, a_curr * phi) <= 1e-12
