"""ctypes front end of the FP64 CPU oracle (``adi_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports it.

All arrays are promoted to contiguous float64 numpy arrays (row-major
``a[j, i]``, x fastest).  The coefficient passed to the oracle is kappa (the
factor of the Laplacian in eq. (f1)); callers holding a speed field pass
``c**2`` computed in FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE arithmetic, no -march)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        path = build()
        l = ctypes.CDLL(path)
        l.oracle_thomas.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        l.oracle_tridiag_batched.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp,
                                             ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int]
        l.oracle_adi_step_parts.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp,
                                            _dp, _dp, ctypes.c_int]
        l.oracle_adi_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, _dp, _dp, _dp, ctypes.c_int, _ip,
                                     _dp, ctypes.c_int, _ip, _dp, ctypes.c_int, ctypes.c_int]
        l.oracle_adi_start.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, _dp, _dp, _dp, ctypes.c_int, _ip,
                                       _dp, ctypes.c_int, _dp, ctypes.c_int]
        l.oracle_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     _dp, _dp, _dp, ctypes.c_int, _ip, _dp, ctypes.c_int, _ip,
                                     _dp, ctypes.c_int, _dp, _dp, ctypes.c_int]
        l.oracle_adi_step_tdc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
        l.oracle_adi_step_split.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
        l.oracle_max_threads.argtypes = []
        for f in (l.oracle_thomas, l.oracle_tridiag_batched, l.oracle_adi_step_parts,
                  l.oracle_adi_run, l.oracle_adi_start, l.oracle_max_threads, l.oracle_adjoint,
                  l.oracle_adi_step_tdc, l.oracle_adi_step_split):
            f.restype = ctypes.c_int
        _lib = l
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


def _iptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_ip)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def thomas(a, b, c, d) -> np.ndarray:
    """Solve one tridiagonal system a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k]."""
    a, b, c, d = (_f64(v) for v in (a, b, c, d))
    x = np.empty_like(d)
    _check(lib().oracle_thomas(int(d.size), _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(x)),
           "thomas")
    return x


def tridiag_batched(a, b, c, d, n: int, batch: int, sys_stride: int, elem_stride: int,
                    threads: int = 0) -> np.ndarray:
    """Batched Thomas over flat arrays with the given strides; returns the solved copy of d."""
    a, b, c = (_f64(v).ravel() for v in (a, b, c))
    x = _f64(d).ravel().copy()
    _check(lib().oracle_tridiag_batched(n, batch, _ptr(a), _ptr(b), _ptr(c), _ptr(x),
                                        sys_stride, elem_stride, threads), "tridiag_batched")
    return x


def _kappa(kappa, nx, ny) -> np.ndarray:
    if np.isscalar(kappa):
        return np.full((ny, nx), float(kappa))
    k = _f64(kappa)
    assert k.shape == (ny, nx)
    return k


def step_parts(kappa, u_prev, u_curr, h: float, dt: float, f=None, threads: int = 0):
    """One step; returns dict with rho, w, d (the ADI increment) and u_next."""
    u_prev, u_curr = _f64(u_prev), _f64(u_curr)
    ny, nx = u_curr.shape
    k = _kappa(kappa, nx, ny)
    f = None if f is None else _f64(f)
    out = {n: np.empty_like(u_curr) for n in ("rho", "w", "d", "u_next")}
    _check(lib().oracle_adi_step_parts(nx, ny, h, dt, _ptr(k), _ptr(u_prev), _ptr(u_curr),
                                       _ptr(f), _ptr(out["rho"]), _ptr(out["w"]),
                                       _ptr(out["d"]), _ptr(out["u_next"]), threads),
           "step_parts")
    return out


def step_tdc(kappa_prev, kappa_next, u_prev, u_curr, h: float, dt: float, f=None, threads: int = 0):
    """One step of eq. (CN1) with a time-dependent coefficient: kappa_prev multiplies the
    Laplacian of u^{k-1}, kappa_next that of u^{k+1}.  Returns u^{k+1}."""
    u_prev, u_curr = _f64(u_prev), _f64(u_curr)
    ny, nx = u_curr.shape
    kp, kn = _kappa(kappa_prev, nx, ny), _kappa(kappa_next, nx, ny)
    f = None if f is None else _f64(f)
    out = np.empty_like(u_curr)
    _check(lib().oracle_adi_step_tdc(nx, ny, h, dt, _ptr(kp), _ptr(kn), _ptr(u_prev), _ptr(u_curr),
                                     _ptr(f), _ptr(out), threads), "step_tdc")
    return out


SPLIT_MODES = {"fr": 1, "theta1": 2}


def step_split(kappa, u_half, u_curr, h: float, dt: float, f=None, f_half=None, mode: str = "fr",
               threads: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """One pair of sub-steps of the split as printed: mode "fr" = eqs. (fr1)-(fr2),
    "theta1" = the line systems of Listing 1.  From (u^{k-1/2}, u^k) returns
    (u^{k+1/2}, u^{k+1}); f is f^k (x-sub-step), f_half is f^{k+1/2} (y-sub-step)."""
    u_half, u_curr = _f64(u_half), _f64(u_curr)
    ny, nx = u_curr.shape
    k = _kappa(kappa, nx, ny)
    f = None if f is None else _f64(f)
    f_half = None if f_half is None else _f64(f_half)
    out_half, out = np.empty_like(u_curr), np.empty_like(u_curr)
    _check(lib().oracle_adi_step_split(nx, ny, h, dt, _ptr(k), SPLIT_MODES[mode], _ptr(u_half),
                                       _ptr(u_curr), _ptr(f), _ptr(f_half), _ptr(out_half), _ptr(out),
                                       threads), "step_split")
    return out_half, out


def run(kappa, u_prev, u_curr, h: float, dt: float, nsteps: int,
        src_idx=None, src_amp=None, rec_idx=None, threads: int = 0
        ) -> Tuple[np.ndarray, np.ndarray, Optional[np.ndarray]]:
    """nsteps ADI steps from (u^{n-1}, u^n); returns (u^{n+nsteps-1}, u^{n+nsteps}, traces)."""
    up = _f64(u_prev).copy()
    uc = _f64(u_curr).copy()
    ny, nx = uc.shape
    k = _kappa(kappa, nx, ny)
    nsrc = 0 if src_idx is None else int(np.asarray(src_idx).size)
    nrec = 0 if rec_idx is None else int(np.asarray(rec_idx).size)
    si = None if nsrc == 0 else np.ascontiguousarray(np.asarray(src_idx, dtype=np.int32))
    sa = None if nsrc == 0 else _f64(src_amp).reshape(-1)
    if nsrc:
        assert sa.size >= nsteps * nsrc
    ri = None if nrec == 0 else np.ascontiguousarray(np.asarray(rec_idx, dtype=np.int32))
    tr = None if nrec == 0 else np.zeros((nsteps, nrec))
    _check(lib().oracle_adi_run(nx, ny, h, dt, _ptr(k), _ptr(up), _ptr(uc), nsrc, _iptr(si),
                                _ptr(sa), nrec, _iptr(ri), _ptr(tr), nsteps, threads), "run")
    return up, uc, tr


def start(kappa, u0, h: float, dt: float, psi=None, mode: str = "ghost",
          src_idx=None, src_amp0=None, threads: int = 0) -> np.ndarray:
    """Level u^1 from u^0 (eq. (CN2) for mode='paper'; second-order ghost start for 'ghost')."""
    u0 = _f64(u0)
    ny, nx = u0.shape
    k = _kappa(kappa, nx, ny)
    psi = None if psi is None else _f64(psi)
    nsrc = 0 if src_idx is None else int(np.asarray(src_idx).size)
    si = None if nsrc == 0 else np.ascontiguousarray(np.asarray(src_idx, dtype=np.int32))
    sa = None if nsrc == 0 else _f64(src_amp0).reshape(-1)
    u1 = np.empty_like(u0)
    m = {"paper": 0, "ghost": 1}[mode]
    _check(lib().oracle_adi_start(nx, ny, h, dt, _ptr(k), _ptr(u0), _ptr(psi), nsrc,
                                  _iptr(si), _ptr(sa), m, _ptr(u1), threads), "start")
    return u1


def initial_levels(prob, threads: int = 0):
    """(u_prev, u_curr, first_level) for a workloads.Problem, in FP64."""
    if prob.u_curr is not None:
        return _f64(prob.u_prev), _f64(prob.u_curr), prob.first_level
    k = prob.kappa_field()
    u0 = _f64(prob.u0)
    u1 = start(k, u0, prob.h, prob.dt, psi=prob.psi, mode=prob.start_mode, threads=threads)
    return u0, u1, 1


def run_problem(prob, nsteps: Optional[int] = None, threads: int = 0):
    """Run a workloads.Problem from its initial levels; returns (u_prev, u_curr, traces)."""
    nsteps = prob.nsteps if nsteps is None else nsteps
    up, uc, _ = initial_levels(prob, threads)
    amp = None if prob.src_amp is None else np.asarray(prob.src_amp)[:nsteps]
    return run(prob.kappa_field(), up, uc, prob.h, prob.dt, nsteps,
               src_idx=prob.src_idx if prob.src_idx.size else None, src_amp=amp,
               rec_idx=prob.rec_idx if prob.rec_idx.size else None, threads=threads)


def adjoint(kappa, u_prev, u_curr, h: float, dt: float, nsteps: int, grad_traces,
            rec_idx, src_idx=None, src_amp=None, threads: int = 0):
    """Reverse pass of `run`: given dJ/d(traces) (nsteps x nrec), returns
    (dJ/dkappa (ny, nx), dJ/d(source values) (nsteps, nsrc) or None)."""
    up, uc = _f64(u_prev), _f64(u_curr)
    ny, nx = uc.shape
    k = _kappa(kappa, nx, ny)
    nsrc = 0 if src_idx is None else int(np.asarray(src_idx).size)
    si = None if nsrc == 0 else np.ascontiguousarray(np.asarray(src_idx, dtype=np.int32))
    sa = None if nsrc == 0 else _f64(src_amp).reshape(-1)
    ri = np.ascontiguousarray(np.asarray(rec_idx, dtype=np.int32))
    gt = _f64(grad_traces).reshape(-1)
    assert gt.size == nsteps * ri.size
    gk = np.zeros((ny, nx))
    ga = None if nsrc == 0 else np.zeros((nsteps, nsrc))
    _check(lib().oracle_adjoint(nx, ny, h, dt, _ptr(k), _ptr(up), _ptr(uc), nsrc, _iptr(si),
                                _ptr(sa), int(ri.size), _iptr(ri), _ptr(gt), nsteps, _ptr(gk),
                                _ptr(ga), threads), "adjoint")
    return gk, ga
