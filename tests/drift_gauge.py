"""Drift gauge: the oracle's forward run and reverse (adjoint) pass transcribed in
numpy for a chosen floating-point type.

TEST INFRASTRUCTURE ONLY.  It measures how much rounding alone moves the
receiver misfit gradient of the same recurrence: run in float64 it follows the
oracle's operation order (no fused multiply-adds, the same association), so it
agrees with the oracle to the last bits; run in float32 every operation rounds to
float32, which is the inherent drift of a correctly rounded single-precision run
of the scheme of eq. (CN1), factored as in eqs. (fr1)-(fr2), and of its discrete
adjoint.  An optional random perturbation of every rounded result by a relative
amount of at most 2^-p (Monte Carlo arithmetic at p bits) measures the same
sensitivity at any precision, float64 included.

Meant for small grids: the line solves run one node at a time along the line,
vectorised over the lines.
"""
from __future__ import annotations

import numpy as np


class _Arith:
    """Rounding of every result to the working type, optionally randomised."""

    def __init__(self, dtype, mca_bits=None, seed=0):
        self.dt = np.dtype(dtype)
        self.rng = None if mca_bits is None else np.random.default_rng(seed)
        self.eps = None if mca_bits is None else 2.0 ** (-mca_bits)

    def __call__(self, x):
        x = np.asarray(x, dtype=self.dt)
        if self.rng is None:
            return x
        return (x * (1.0 + self.eps * self.rng.uniform(-1.0, 1.0, x.shape))).astype(self.dt)

    def c(self, v):
        """A scalar constant of the working type (computed in float64, rounded once)."""
        return self.dt.type(v)


def _thomas_lines(R, a, b, c, d):
    """Thomas along axis 0 of (n, lines) arrays: a x[k-1] + b x[k] + c x[k+1] = d."""
    n = d.shape[0]
    cp = np.empty_like(d)
    dp = np.empty_like(d)
    cp[0] = R(c[0] / b[0])
    dp[0] = R(d[0] / b[0])
    for k in range(1, n):
        piv = R(b[k] - R(a[k] * cp[k - 1]))
        cp[k] = R(c[k] / piv)
        dp[k] = R(R(d[k] - R(a[k] * dp[k - 1])) / piv)
    x = np.empty_like(d)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = R(dp[k] - R(cp[k] * x[k + 1]))
    return x


def _shift(v, axis, step):
    """v at the neighbour step (+1 / -1) along axis, zero beyond the walls."""
    out = np.zeros_like(v)
    if axis == 1:
        if step > 0:
            out[:, :-1] = v[:, 1:]
        else:
            out[:, 1:] = v[:, :-1]
    else:
        if step > 0:
            out[:-1, :] = v[1:, :]
        else:
            out[1:, :] = v[:-1, :]
    return out


def _lxx(R, v, ih2):
    return R(R(R(_shift(v, 1, -1) - R(R.c(2.0) * v)) + _shift(v, 1, 1)) * ih2)


def _lyy(R, v, ih2):
    return R(R(R(_shift(v, 0, -1) - R(R.c(2.0) * v)) + _shift(v, 0, 1)) * ih2)


def _lap(R, v, ih2):
    return R(_lxx(R, v, ih2) + _lyy(R, v, ih2))


def _solves(R, off, rhs, transposed=False):
    """(I - beta K Lxx) w = rhs on every x-line, then (I - beta K Lyy) d = w on every
    y-line (transposed=False).  transposed=True: the transposed y-lines, then the
    transposed x-lines (rows -off_{k-1}, 1 + 2 off_k, -off_{k+1}); returns both stages."""
    one, two = R.c(1.0), R.c(2.0)
    diag = R(one + R(two * off))

    def along(axis, v):
        # lines along `axis`; move the line axis first
        o = off if axis == 0 else off.T
        dg = diag if axis == 0 else diag.T
        vv = v if axis == 0 else v.T
        if transposed:
            lo = np.zeros_like(o)
            lo[1:] = -o[:-1]
            hi = np.zeros_like(o)
            hi[:-1] = -o[1:]
        else:
            lo, hi = -o, -o
        x = _thomas_lines(R, lo, dg, hi, np.ascontiguousarray(vv))
        return x if axis == 0 else x.T

    if not transposed:
        w = along(1, rhs)
        return w, along(0, w)
    nu = along(0, rhs)
    return nu, along(1, nu)


def misfit_gradient(kappa, u_prev, u_curr, h, dt, nsteps, src_idx, src_amp, rec_idx, target,
                    dtype=np.float64, mca_bits=None, seed=0):
    """Forward run with receivers, misfit J = sum (tr - target)^2, then the reverse pass.

    Returns (dJ/dkappa (ny, nx), dJ/d(source value) (nsteps, nsrc), traces), all computed
    in `dtype` (inputs are rounded to it once).  Same recurrences as the oracle:
      forward   rho = dt^2 (kappa Lap u^k + f^k), A_x w = rho, A_y d = w,
                u^{k+1} = 2 u^k - u^{k-1} + d;
      reverse   nu = A_y^{-T} lambda^{k+1}, mu = A_x^{-T} nu,
                dJ/dkappa += dt^2 mu Lap u^k + beta (mu Lxx w^k + nu Lyy d^k),
                dJ/df^k = dt^2 mu at the sources,
                lambda^k = g^k + 2 lambda^{k+1} - lambda^{k+2} + dt^2 Lap(kappa mu)."""
    R = _Arith(dtype, mca_bits, seed)
    ny, nx = np.shape(u_curr)
    kap = np.asarray(kappa, dtype=R.dt)
    if kap.ndim == 0:
        kap = np.full((ny, nx), kap, dtype=R.dt)
    ih2 = R.c(1.0 / (h * h))
    tau2 = R.c(dt * dt)
    beta = R.c(0.5 * dt * dt)
    s = R.c(0.5 * dt * dt / (h * h))
    off = R(s * kap)
    si = np.asarray(src_idx, dtype=np.int64).ravel()
    ri = np.asarray(rec_idx, dtype=np.int64).ravel()
    amp = np.asarray(src_amp, dtype=R.dt).reshape(nsteps, si.size)
    U = [np.asarray(u_prev, dtype=R.dt).copy(), np.asarray(u_curr, dtype=R.dt).copy()]
    W, D = [None], [None]
    tr = np.zeros((nsteps, ri.size), dtype=R.dt)
    for k in range(1, nsteps + 1):
        f = np.zeros(nx * ny, dtype=R.dt)
        np.add.at(f, si, amp[k - 1])
        rho = R(tau2 * R(R(kap * _lap(R, U[k], ih2)) + f.reshape(ny, nx)))
        w, d = _solves(R, off, rho)
        W.append(w)
        D.append(d)
        U.append(R(R(R(R.c(2.0) * U[k]) - U[k - 1]) + d))
        tr[k - 1] = U[k + 1].ravel()[ri]
    gtr = R(R.c(2.0) * R(tr - np.asarray(target, dtype=R.dt)))
    gk = np.zeros((ny, nx), dtype=R.dt)
    ga = np.zeros((nsteps, si.size), dtype=R.dt)
    lam2 = np.zeros((ny, nx), dtype=R.dt)
    lam1 = np.zeros(nx * ny, dtype=R.dt)
    np.add.at(lam1, ri, gtr[nsteps - 1])
    lam1 = lam1.reshape(ny, nx)
    for k in range(nsteps, 0, -1):
        nu, mu = _solves(R, off, lam1, transposed=True)
        gk = R(gk + R(tau2 * R(mu * _lap(R, U[k], ih2))))
        gk = R(gk + R(beta * R(R(mu * _lxx(R, W[k], ih2)) + R(nu * _lyy(R, D[k], ih2)))))
        ga[k - 1] = R(tau2 * mu.ravel()[si])
        lk = R(R(R(R.c(2.0) * lam1) - lam2) + R(tau2 * _lap(R, R(kap * mu), ih2)))
        lam2 = lam1
        lam1 = lk
        if k >= 2:
            flat = lam1.ravel().copy()
            np.add.at(flat, ri, gtr[k - 2])
            lam1 = flat.reshape(ny, nx)
    return gk, ga, tr


def run(kappa, u_prev, u_curr, h, dt, nsteps, dtype=np.float64):
    """The oracle's forward run (no sources) in `dtype`: returns u^{n+nsteps}."""
    R = _Arith(dtype)
    ny, nx = np.shape(u_curr)
    kap = np.asarray(kappa, dtype=R.dt)
    if kap.ndim == 0:
        kap = np.full((ny, nx), kap, dtype=R.dt)
    ih2 = R.c(1.0 / (h * h))
    tau2 = R.c(dt * dt)
    off = R(R.c(0.5 * dt * dt / (h * h)) * kap)
    um = np.asarray(u_prev, dtype=R.dt).copy()
    uc = np.asarray(u_curr, dtype=R.dt).copy()
    for _ in range(nsteps):
        rho = R(tau2 * R(kap * _lap(R, uc, ih2)))
        _, d = _solves(R, off, rho)
        um, uc = uc, R(R(R(R.c(2.0) * uc) - um) + d)
    return uc
