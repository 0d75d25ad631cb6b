"""The split as printed on the GPU (paper-fidelity modes): eqs. (fr1)-(fr2) and
Listing 1's line systems, one pair of sub-steps per call, against the oracle's
step_split (FP64 <= 1e-12, FP32 <= 1e-5 relative L2 after the run), with a
per-node kappa, point sources in both sub-steps and receivers."""
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


@pytest.mark.parametrize("mode", ["fr", "theta1"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", [(120, 90), (33, 300), (257, 64), (1, 7)])
def test_split_matches_oracle(adw, oracle_lib, mode, dtype, nx, ny):
    npd = np.float32 if dtype == "f32" else np.float64
    tdt = torch.float32 if dtype == "f32" else torch.float64
    h = 1.0 / (max(nx, ny) + 1)
    dt = 0.4 * h / 2.0
    c = wl.smooth_field(nx, ny, 1.0, 2.0, seed=nx + ny).astype(npd)
    kap = c.astype(np.float64) ** 2
    npairs = 20
    u0 = wl.gaussian_pulse(nx, ny, sigma=0.1).astype(npd)
    uh, uc = u0.copy(), (0.995 * u0).astype(npd)
    src = np.array([(ny // 2) * nx + nx // 3], np.int32)
    rng = np.random.default_rng(nx)
    amp = (rng.standard_normal((npairs, 1)) * 20.0).astype(npd)
    amp_h = (rng.standard_normal((npairs, 1)) * 20.0).astype(npd)
    rec = np.array([0, (ny // 3) * nx + nx // 2, nx * ny - 1], np.int32)
    print(f"split {mode} {dtype} {nx}x{ny}", flush=True)

    wave = adw.Wave(nx, ny, h, dt, c=dev(c), dtype=tdt)
    a, b = dev(uh), dev(uc)
    traces = torch.zeros((npairs, rec.size), dtype=tdt, device="cuda")
    for k in range(npairs):
        a, b = wave.step_split(a, b, mode=mode, src_idx=dev(src), src_amp=dev(amp[k]),
                               src_amp_half=dev(amp_h[k]), rec_idx=dev(rec), traces=traces[k])
    torch.cuda.synchronize()
    got_h, got, gtr = a.cpu().numpy(), b.cpu().numpy(), traces.cpu().numpy()
    wave.close()

    rh, rc = uh.astype(np.float64), uc.astype(np.float64)
    rtr = np.zeros((npairs, rec.size))
    for k in range(npairs):
        f = np.zeros((ny, nx))
        fh = np.zeros((ny, nx))
        f.ravel()[src] += amp[k]
        fh.ravel()[src] += amp_h[k]
        rh, rc = oracle_lib.step_split(kap, rh, rc, h, dt, f=f, f_half=fh, mode=mode)
        rtr[k] = rc.ravel()[rec]
    assert rel_l2(got, rc) <= TOL[dtype]
    assert rel_l2(got_h, rh) <= TOL[dtype]
    assert rel_l2(gtr, rtr) <= TOL[dtype]


def test_split_rejects_bad_arguments(adw):
    w = adw.Wave(16, 16, 1.0 / 17, 0.5 / 17, c=1.0, dtype=torch.float64)
    a = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(KeyError):
        w.step_split(a, a.clone(), mode="other")
    with pytest.raises(RuntimeError):
        w.step_split(a, a, mode="fr")
    w.close()
