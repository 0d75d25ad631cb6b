"""Steps of eq. (CN1) with a time-dependent coefficient on the GPU, against the
oracle's step (FP64 <= 1e-12, FP32 <= 1e-5 relative L2 after the run), with a
per-node kappa(t, x, y), point sources and receivers; and for a coefficient
constant in time, the plain step."""
import math

import numpy as np
import pytest

from tests.conftest import rel_l2
from paper_2006_10142_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def adw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2006_10142_amd as m
    m._lib.load()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", [(120, 90), (257, 64), (33, 300)])
def test_time_dependent_steps_match_oracle(adw, oracle_lib, dtype, nx, ny):
    npd = np.float32 if dtype == "f32" else np.float64
    tdt = torch.float32 if dtype == "f32" else torch.float64
    h = 1.0 / (max(nx, ny) + 1)
    dt = 0.4 * h / 2.0
    ka = wl.smooth_field(nx, ny, 1.0, 3.0, seed=nx)
    kb = wl.smooth_field(nx, ny, 0.0, 1.0, seed=ny)
    kap = lambda t: (ka + 0.8 * math.sin(40.0 * t) * kb).astype(npd)   # rounded once per level
    nsteps = 20
    u0 = wl.gaussian_pulse(nx, ny, sigma=0.1).astype(npd)
    up, uc = u0.copy(), (0.999 * u0).astype(npd)
    src = np.array([(ny // 2) * nx + nx // 3], np.int32)
    amp = (np.random.default_rng(3).standard_normal((nsteps, 1)) * 30.0).astype(npd)
    rec = np.array([5, (ny // 4) * nx + nx // 2, nx * ny - 3], np.int32)
    print(f"tdc {dtype} {nx}x{ny}", flush=True)

    wave = adw.Wave(nx, ny, h, dt, kappa=dev(kap(0.0)), dtype=tdt)
    a, b = dev(up), dev(uc)
    traces = torch.zeros((nsteps, rec.size), dtype=tdt, device="cuda")
    for k in range(nsteps):
        t = (k + 1) * dt
        a, b = wave.step_tdc(a, b, kappa_prev=dev(kap(t - dt)), kappa_next=dev(kap(t + dt)),
                             src_idx=dev(src), src_amp=dev(amp[k]), rec_idx=dev(rec), traces=traces[k])
    torch.cuda.synchronize()
    got, gtr = b.cpu().numpy(), traces.cpu().numpy()
    info = wave.info()
    wave.close()

    rp, rc = up.astype(np.float64), uc.astype(np.float64)
    rtr = np.zeros((nsteps, rec.size))
    for k in range(nsteps):
        t = (k + 1) * dt
        f = np.zeros((ny, nx))
        f.ravel()[src] += amp[k]
        rp, rc = rc, oracle_lib.step_tdc(kap(t - dt), kap(t + dt), rp, rc, h, dt, f=f)
        rtr[k] = rc.ravel()[rec]
    assert rel_l2(got, rc) <= TOL[dtype]
    assert rel_l2(gtr, rtr) <= TOL[dtype]
    assert info["fused_step"] == 0


def test_constant_coefficient_is_the_plain_step(adw):
    nx, ny = 150, 97
    h = 1.0 / 151
    dt = 0.5 * h
    kap = wl.smooth_field(nx, ny, 1.0, 4.0, seed=2)
    u0 = wl.gaussian_pulse(nx, ny, sigma=0.12)
    w1 = adw.Wave(nx, ny, h, dt, kappa=dev(kap), dtype=torch.float64)
    w2 = adw.Wave(nx, ny, h, dt, kappa=dev(kap), dtype=torch.float64)
    a1, b1 = dev(u0), dev(0.99 * u0)
    a2, b2 = a1.clone(), b1.clone()
    for _ in range(15):
        a1, b1 = w1.step_tdc(a1, b1)
    a2, b2 = w2.step(a2, b2, 15)
    torch.cuda.synchronize()
    assert rel_l2(b1.cpu().numpy(), b2.cpu().numpy()) <= 1e-14
    w1.close()
    w2.close()


def test_set_kappa_restores_the_one_pass_step(adw):
    n = 512
    w = adw.Wave(n, n, 1.0 / (n + 1), 0.5 / (n + 1), c=1.0, dtype=torch.float32)
    assert w.info()["fused_step"] == 1
    a, b = torch.zeros((n, n), device="cuda"), torch.zeros((n, n), device="cuda")
    k = torch.ones((n, n), device="cuda")
    a, b = w.step_tdc(a, b, kappa_prev=k, kappa_next=k)
    assert w.info()["fused_step"] == 0 and w.info()["fused_allowed"] == 0
    w.set_kappa(k)
    assert w.info()["fused_step"] == 1
    w.close()
