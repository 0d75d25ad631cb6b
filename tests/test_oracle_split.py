"""Pins of the oracle's split as printed: eqs. (fr1)-(fr2) ("fr", weights 1/2 on the
new and the oldest level of each sub-step) and the line systems of Listing 1
("theta1": a = c = tau^2, b = 2 tau^2 + h^2, weight 1 on the new level only).

  * each sub-step against its printed equation solved densely with Kronecker
    operators and a per-node kappa (x-sub-step with f^k first, then the y-sub-step
    with f^{k+1/2});
  * the scalar recurrence of a grid mode under a constant kappa, over many steps;
  * the reason the split is not the scheme used elsewhere: the printed split moves
    a smooth mode sqrt(2) times faster than the continuous wave, while the
    factored step of eq. (CN1) moves it at the right speed."""
import math

import numpy as np
import pytest

from tests.conftest import rel_l2
from tests.test_oracle_pins import dense_ops

THETA = {"fr": (0.5, 0.5), "theta1": (1.0, 0.0)}


def grid(nx, ny, h):
    x = (np.arange(nx) + 1) * h
    y = (np.arange(ny) + 1) * h
    return np.meshgrid(x, y)


def dense_pair(kap, u_half, u_curr, f, f_half, h, dt, mode):
    """(u_new - 2 u_mid + u_old)/dt^2 - tn K D u_new - to K D u_old = f, D = Lxx then Lyy."""
    ny, nx = u_curr.shape
    Lx, Ly = dense_ops(nx, ny, h)
    K = np.diag(kap.ravel())
    tn, to = THETA[mode]
    n = nx * ny
    I = np.eye(n)

    def sub(D, u_old, u_mid, g):
        A = I / dt ** 2 - tn * K @ D
        rhs = (2 * u_mid.ravel() - u_old.ravel()) / dt ** 2 + to * K @ D @ u_old.ravel() + g.ravel()
        return np.linalg.solve(A, rhs).reshape(ny, nx)

    uh = sub(Lx, u_half, u_curr, f)
    return uh, sub(Ly, u_curr, uh, f_half)


@pytest.mark.parametrize("mode", ["fr", "theta1"])
@pytest.mark.parametrize("nx,ny", [(7, 5), (1, 6), (9, 1)])
def test_pair_matches_printed_equations(oracle_lib, mode, nx, ny):
    rng = np.random.default_rng(nx * 10 + ny)
    h, dt = 1.0 / (max(nx, ny) + 1), 0.37 / (max(nx, ny) + 1)
    kap = rng.uniform(1.0, 4.0, (ny, nx))
    u_half, u_curr, f, fh = (rng.standard_normal((ny, nx)) for _ in range(4))
    got_h, got = oracle_lib.step_split(kap, u_half, u_curr, h, dt, f=f, f_half=fh, mode=mode)
    ref_h, ref = dense_pair(kap, u_half, u_curr, f, fh, h, dt, mode)
    assert rel_l2(got_h, ref_h) <= 1e-13
    assert rel_l2(got, ref) <= 1e-13


def test_modes_differ_and_sub_steps_are_ordered(oracle_lib):
    """Swapping the sub-step order, or the two modes, gives a different answer."""
    rng = np.random.default_rng(3)
    nx, ny, h, dt = 8, 6, 1.0 / 9, 0.05
    kap = rng.uniform(1.0, 2.0, (ny, nx))
    uh, uc = rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx))
    a = oracle_lib.step_split(kap, uh, uc, h, dt, mode="fr")[1]
    b = oracle_lib.step_split(kap, uh, uc, h, dt, mode="theta1")[1]
    swapped = oracle_lib.step_split(kap.T.copy(), uh.T.copy(), uc.T.copy(), h, dt, mode="fr")[1].T
    assert rel_l2(a, b) > 1e-3
    assert rel_l2(a, swapped) > 1e-3


@pytest.mark.parametrize("mode", ["fr", "theta1"])
def test_mode_recurrence(oracle_lib, mode):
    """u = a sin(p pi x) sin(q pi y): D multiplies the mode by -lam, so each sub-step is
    a_new (1 + tn dt^2 kappa lam) = 2 a_mid - a_old (1 + to dt^2 kappa lam)."""
    n, p, q = 30, 2, 3
    h = 1.0 / (n + 1)
    dt = 0.8 * h
    kappa = 2.5
    X, Y = grid(n, n, h)
    phi = np.sin(p * math.pi * X) * np.sin(q * math.pi * Y)
    lx = 4.0 * math.sin(p * math.pi * h / 2) ** 2 / h ** 2
    ly = 4.0 * math.sin(q * math.pi * h / 2) ** 2 / h ** 2
    tn, to = THETA[mode]
    a_half, a = 1.0, 0.97
    uh, uc = a_half * phi, a * phi
    for _ in range(150):
        uh, uc = oracle_lib.step_split(np.full_like(phi, kappa), uh, uc, h, dt, mode=mode)
        a_new_half = (2 * a - a_half * (1 + to * dt * dt * kappa * lx)) / (1 + tn * dt * dt * kappa * lx)
        a_new = (2 * a_new_half - a * (1 + to * dt * dt * kappa * ly)) / (1 + tn * dt * dt * kappa * ly)
        a_half, a = a_new_half, a_new
    # the theta1 system damps the mode: errors are measured against the initial amplitude
    scale = np.linalg.norm(phi)
    assert np.linalg.norm(uc - a * phi) <= 1e-12 * scale
    assert np.linalg.norm(uh - a_half * phi) <= 1e-12 * scale
    if mode == "fr":
        assert abs(a) > 0.1                       # the printed split conserves the mode's energy
    else:
        assert abs(a) < 1e-3                      # Listing 1's system is dissipative


def _period_in_steps(levels):
    """mean distance between sign changes of a sampled oscillation, times two"""
    s = np.sign(levels)
    idx = np.nonzero(s[1:] * s[:-1] < 0)[0]
    # linear interpolation of each crossing
    t = idx + levels[idx] / (levels[idx] - levels[idx + 1])
    return 2.0 * np.mean(np.diff(t))


def test_printed_split_is_sqrt2_too_fast(oracle_lib):
    """Lowest mode, kappa = 1: the continuous period is 2 / sqrt(2) = sqrt(2).  The
    printed split's mode completes a period sqrt(2) times sooner; the factored step of
    eq. (CN1) keeps the continuous period (both to O(dt^2 + h^2))."""
    n = 31
    h = 1.0 / (n + 1)
    dt = 0.25 * h
    X, Y = grid(n, n, h)
    phi = np.sin(math.pi * X) * np.sin(math.pi * Y)
    kap = np.ones_like(phi)
    nsteps = 1200
    uh, uc = phi.copy(), phi.copy()
    amp = []
    for _ in range(nsteps):
        uh, uc = oracle_lib.step_split(kap, uh, uc, h, dt, mode="fr")
        amp.append(float(np.vdot(uc.ravel(), phi.ravel())))
    split_period = _period_in_steps(np.array(amp)) * dt
    up, uc2 = phi.copy(), phi * math.cos(math.sqrt(2) * math.pi * dt)
    amp2 = []
    for _ in range(nsteps):
        up, uc2 = uc2, oracle_lib.step_parts(kap, up, uc2, h, dt)["u_next"]
        amp2.append(float(np.vdot(uc2.ravel(), phi.ravel())))
    scheme_period = _period_in_steps(np.array(amp2)) * dt
    exact = 2.0 / math.sqrt(2.0)
    assert abs(exact / split_period - math.sqrt(2)) < 5e-3, split_period
    assert abs(scheme_period / exact - 1.0) < 5e-3, scheme_period
