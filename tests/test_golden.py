"""The stored reference values in tests/golden against the oracle, and against
what fixes them independently of it: the discrete closed form of the standing
wave, and the residual of each stored tridiagonal solution."""
import math

import numpy as np

from tests.conftest import rel_l2
from tests.golden import cases, store
from paper_2006_10142_amd import workloads as wl


def test_oracle_reproduces_the_stored_runs(oracle_lib):
    for name, make in cases.CASES.items():
        p, nodes = make()
        offs, vals, recs, traces = store.load(name)
        assert np.array_equal(offs, nodes), name
        _, uc, tr = oracle_lib.run_problem(p)
        assert rel_l2(uc.ravel()[offs], vals) <= 1e-14, name
        if traces is not None:
            assert np.array_equal(recs, p.rec_idx), name
            assert np.abs(traces).max() > 1e-3, name          # the wave reached the receivers
            assert rel_l2(tr, traces) <= 1e-14, name


def test_stored_standing_wave_is_the_discrete_closed_form():
    """u^(n) = cos(n theta) sin(pi x) sin(pi y), cos(theta) = 1 - g/2, with the 1-D
    eigenvalue lam = 4 sin^2(pi h / 2) / h^2 of each axis (kappa = 1):
    g = dt^2 2 lam / (1 + beta lam)^2, beta = dt^2 / 2.  The stored level is u^(201)."""
    p, _ = cases.c1_standing_wave()
    offs, vals, _, _ = store.load("c1_standing_wave_128_f64")
    lam = 4 * math.sin(math.pi * p.h / 2) ** 2 / p.h ** 2
    beta = p.dt ** 2 / 2
    g = p.dt ** 2 * 2 * lam / (1 + beta * lam) ** 2
    theta = math.acos(1 - g / 2)
    exact = math.cos((p.nsteps + 1) * theta) * wl.sine_mode(p.nx, p.ny).ravel()[offs]
    assert rel_l2(vals, exact) <= 1e-12


def test_stored_tridiagonal_solutions_satisfy_their_systems():
    for rows in store.load_tridiag():
        a, b, c, d, x = rows.T
        n = x.size
        lhs = b * x
        lhs[1:] += a[1:] * x[:-1]
        lhs[:-1] += c[:-1] * x[1:]
        assert np.abs(lhs - d).max() <= 1e-14 * max(1.0, np.abs(d).max())
        assert n in (1, 2, 7, 33)


def test_oracle_reproduces_the_stored_tridiagonal_solutions(oracle_lib):
    for rows in store.load_tridiag():
        a, b, c, d, x = rows.T
        assert np.array_equal(oracle_lib.thomas(a, b, c, d), x)
