"""The cyclic-reduction line solver (the paper's Sec. 3.1 algorithm, one launch per
level for all lines of a sweep), kept as a same-GPU baseline: it must give the
oracle's answer to the same bars as the default solvers (FP64 <= 1e-12, FP32
<= 1e-5 relative L2 after the run), on line lengths that are and are not of the
form 2^m - 1, with sources and receivers."""
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


def run_case(adw, oracle_lib, nx, ny, dtype, nsteps=12, seed=1, cr=True):
    npd = np.float32 if dtype == "f32" else np.float64
    tdt = torch.float32 if dtype == "f32" else torch.float64
    h = 1.0 / (max(nx, ny) + 1)
    c = wl.smooth_field(nx, ny, 1.0, 3.0, seed=seed).astype(npd)
    dt = 0.5 * h / 3.0
    u0 = wl.gaussian_pulse(nx, ny, sigma=0.15).astype(npd)
    rng = np.random.default_rng(seed)
    src = np.array([(ny // 2) * nx + nx // 3, (ny - 1) * nx + nx - 1], np.int32)
    amp = (rng.standard_normal((nsteps, 2)) * 20.0).astype(npd)
    rec = np.array([0, (ny // 3) * nx + nx // 2, nx * ny - 1], np.int32)
    wave = adw.Wave(nx, ny, h, dt, c=dev(c), dtype=tdt)
    a = dev(u0)
    b = wave.start(a)
    wave.set_tuning(cyclic_reduction=cr)
    info = wave.info()
    tr = torch.zeros((nsteps, rec.size), dtype=tdt, device="cuda")
    a, b = wave.step(a, b, nsteps, src_idx=dev(src), src_amp=dev(amp), rec_idx=dev(rec), traces=tr)
    torch.cuda.synchronize()
    got, gtr = b.cpu().numpy(), tr.cpu().numpy()
    wave.close()
    kap = c.astype(np.float64) ** 2
    u1 = oracle_lib.start(kap, u0, h, dt)
    _, ref, rtr = oracle_lib.run(kap, u0, u1, h, dt, nsteps, src_idx=src, src_amp=amp, rec_idx=rec)
    return got, gtr, ref, rtr, info


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", [(1, 1), (5, 3), (7, 15), (100, 63), (127, 128), (300, 211), (1024, 17)])
def test_cyclic_reduction_matches_oracle(adw, oracle_lib, dtype, nx, ny):
    print(f"cr {dtype} {nx}x{ny}", flush=True)
    got, gtr, ref, rtr, info = run_case(adw, oracle_lib, nx, ny, dtype)
    assert info["line_solver"] == 2
    assert rel_l2(got, ref) <= TOL[dtype]
    assert rel_l2(gtr, rtr) <= TOL[dtype]


def test_cyclic_reduction_switches_back(adw):
    wave = adw.Wave(64, 48, 1.0 / 65, 0.5 / 65, c=1.0, dtype=torch.float64)
    wave.set_tuning(cyclic_reduction=True)
    inf = wave.info()
    m = lambda n: int(np.ceil(np.log2(n + 1)))
    assert inf["line_solver"] == 2 and inf["kernels_per_step"] == 1 + 2 * m(64) + 2 * m(48)
    wave.set_tuning(cyclic_reduction=False)
    assert wave.info()["line_solver"] == 1
    wave.close()
