"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (relative L2 over all interior nodes, computed in FP64):
  FP64 runs  <= 1e-12 after the full run (single line solves and steps <= 1e-13);
  FP32 runs  <= 1e-5 after the full run.
FP32 inputs are rounded once by the workload generators; the oracle consumes
those same values promoted to FP64.
"""
import math

import numpy as np
import pytest

from tests.conftest import max_rel, rel_l2
from paper_2006_10142_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_RUN = {"f64": 1e-12, "f32": 1e-5}
TOL_ONE = {"f64": 1e-13, "f32": 1e-5}


@pytest.fixture(scope="module")
def adw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2006_10142_amd as m
    m._lib.load()
    return m


def tdt(dtype):
    return torch.float32 if dtype == "f32" else torch.float64


def npdt(dtype):
    return np.float32 if dtype == "f32" else np.float64


def dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(tdt(dtype))
    return t.cuda()


def say(msg):
    print(msg, flush=True)


# -------------------------------------------------------- batched solves ----
def dd_systems(rng, size):
    a = rng.uniform(-1, 1, size)
    c = rng.uniform(-1, 1, size)
    b = (np.abs(a) + np.abs(c) + rng.uniform(0.05, 1.0, size)) * rng.choice([-1.0, 1.0], size)
    d = rng.standard_normal(size)
    return a, b, c, d


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,batch", [(1, 5), (2, 9), (3, 33), (37, 33), (64, 7), (128, 5),
                                     (129, 5), (1000, 4), (4097, 3), (8192, 3)])
def test_tridiag_contiguous(adw, oracle_lib, dtype, n, batch):
    say(f"tridiag contiguous {dtype} n={n} batch={batch}")
    rng = np.random.default_rng(n * 31 + batch)
    a, b, c, d = (v.astype(npdt(dtype)) for v in dd_systems(rng, n * batch))
    ref = oracle_lib.tridiag_batched(a, b, c, d, n, batch, n, 1)
    A, B, C, D = (dev(v) for v in (a, b, c, d))
    adw.tridiag_solve_batched(A, B, C, D, n, batch, n, 1)
    torch.cuda.synchronize()
    assert rel_l2(D.cpu().numpy(), ref) <= TOL_ONE[dtype]
    assert np.array_equal(A.cpu().numpy(), a)        # coefficients untouched


STRIDED = {  # layout: (n, batch, sys_stride, elem_stride)
    "interleaved": (300, 257, 1, 257),
    "padded": (77, 19, 3 * 77 + 5, 3),
    "long": (20000, 3, 20000, 1),
    "one_row_tail": (33, 65, 1, 65),      # FP32 chunks of 32: the last chunk is one row
    "one_row_tail_f64": (17, 40, 1, 40),  # FP64 chunks of 16
    "single_chunk": (5, 70, 1, 70),
    "n1": (1, 9, 2, 1),
    "n2": (2, 9, 1, 9),
    "long_strided": (9001, 2, 1, 2),
    # interface systems of 256 (FP32) / 512 (FP64) rows: the parallel interface solve with
    # 16 / 32 threads per system
    "interleaved_8192": (8192, 64, 1, 64),
    # interface systems longer than the parallel solve takes (1250 / 2500 rows): the
    # serial interface solve
    "very_long_strided": (40000, 2, 1, 2),
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", list(STRIDED))
def test_tridiag_strided(adw, oracle_lib, dtype, layout):
    n, batch, ss, es = STRIDED[layout]
    say(f"tridiag {layout} {dtype} n={n} batch={batch}")
    size = (batch - 1) * ss + (n - 1) * es + 1
    rng = np.random.default_rng(5)
    a, b, c, d = (v.astype(npdt(dtype)) for v in dd_systems(rng, size))
    ref = oracle_lib.tridiag_batched(a, b, c, d, n, batch, ss, es)
    A, B, C, D = (dev(v) for v in (a, b, c, d))
    adw.tridiag_solve_batched(A, B, C, D, n, batch, ss, es)
    torch.cuda.synchronize()
    got = D.cpu().numpy()
    assert rel_l2(got, ref) <= TOL_ONE[dtype]
    mask = np.ones(size, bool)
    for s in range(batch):
        mask[s * ss + np.arange(n) * es] = False
    assert np.array_equal(got[mask], d[mask])        # gaps untouched


def test_tridiag_interleaved_full_size(adw, oracle_lib):
    """8192 interleaved FP32 systems of 8192 unknowns (the measured line-solve case):
    sampled systems against the oracle, and the residual of all of them."""
    n = batch = 8192
    say(f"tridiag interleaved full size f32 n={n} batch={batch}")
    g = torch.Generator(device="cuda").manual_seed(11)
    A = torch.rand(n * batch, device="cuda", generator=g) - 0.5
    C = torch.rand(n * batch, device="cuda", generator=g) - 0.5
    B = A.abs() + C.abs() + 0.5
    D0 = torch.rand(n * batch, device="cuda", generator=g)
    D = D0.clone()
    adw.tridiag_solve_batched(A, B, C, D, n, batch, 1, batch)
    torch.cuda.synchronize()
    a, b, c, d, x = (t.view(n, batch) for t in (A, B, C, D0, D))
    res = b * x - d
    res[1:] += a[1:] * x[:-1]
    res[:-1] += c[:-1] * x[1:]
    assert (res.norm() / d.norm()).item() <= 1e-6
    cols = [0, 1, 63, 64, 4095, 8190, 8191]
    sub = [t[:, cols].double().t().contiguous().cpu().numpy().ravel() for t in (a, b, c, d)]
    ref = oracle_lib.tridiag_batched(*sub, n, len(cols), n, 1)
    got = x[:, cols].double().t().contiguous().cpu().numpy().ravel()
    assert rel_l2(got, ref) <= TOL_ONE["f32"]
    del A, B, C, D0, D, a, b, c, d, x, res
    torch.cuda.empty_cache()


# ------------------------------------------------------------- one step ----
SHAPES = [(1, 1), (1, 5), (5, 1), (2, 3), (7, 5), (64, 64), (100, 37), (129, 257),
          (513, 70), (1000, 33), (2049, 40), (4096, 12), (8192, 9)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_single_step_increment(adw, oracle_lib, dtype, nx, ny):
    """u_prev = 2 u_curr makes u^{n+1} equal the ADI increment d exactly."""
    say(f"single step {dtype} {nx}x{ny}")
    rng = np.random.default_rng(nx * 7 + ny)
    h = 1.0 / (max(nx, ny) + 1)
    dt = 0.8 * h
    c = rng.uniform(1.0, 3.0, (ny, nx)).astype(npdt(dtype))
    uc = rng.standard_normal((ny, nx)).astype(npdt(dtype))
    up = (2 * uc.astype(np.float64)).astype(npdt(dtype))
    src_idx = np.array([(ny // 2) * nx + nx // 3], np.int32)
    amp = np.array([[1.0 / (h * h)]], npdt(dtype))
    ref = oracle_lib.step_parts(c.astype(np.float64) ** 2, up, uc, h, dt,
                                f=np.bincount(src_idx, weights=amp[0].astype(np.float64),
                                              minlength=nx * ny).reshape(ny, nx))["d"]
    wave = adw.Wave(nx, ny, h, dt, c=dev(c), dtype=tdt(dtype))
    a, b = dev(up), dev(uc)
    a, b = wave.step(a, b, 1, src_idx=dev(src_idx), src_amp=dev(amp))
    torch.cuda.synchronize()
    assert rel_l2(b.cpu().numpy(), ref) <= TOL_ONE[dtype]


# ------------------------------------------------------------ full runs ----
def gpu_run(adw, prob, nsteps=None, rec=False, fused_step=None):
    nsteps = prob.nsteps if nsteps is None else nsteps
    t = tdt(prob.dtype)
    wave = adw.Wave(prob.nx, prob.ny, prob.h, prob.dt, dtype=t,
                    c=dev(prob.c) if prob.c is not None else prob.c_scalar,
                    kappa=dev(prob.kappa) if prob.kappa is not None else None)
    if fused_step is not None:
        wave.set_tuning(fused_step=fused_step)
        assert wave.info()["fused_step"] == int(fused_step)
    if prob.u_curr is not None:
        a, b = dev(prob.u_prev), dev(prob.u_curr)
    else:
        a = dev(prob.u0)
        b = wave.start(a, psi=None if prob.psi is None else dev(prob.psi), mode=prob.start_mode)
    kw = {}
    if prob.src_amp is not None:
        kw.update(src_idx=dev(prob.src_idx), src_amp=dev(np.asarray(prob.src_amp)[:nsteps]))
    traces = None
    if rec and prob.rec_idx.size:
        traces = torch.zeros((nsteps, prob.rec_idx.size), dtype=t, device="cuda")
        kw.update(rec_idx=dev(prob.rec_idx), traces=traces)
    a, b = wave.step(a, b, nsteps, **kw)
    torch.cuda.synchronize()
    out = (a.cpu().numpy(), b.cpu().numpy(), None if traces is None else traces.cpu().numpy())
    wave.close()
    return out


def test_c1_standing_wave(adw, oracle_lib):
    """C1: 128^2, FP64, ghost start, 200 steps: oracle and discrete closed form."""
    p = wl.config_c1()
    say("C1 f64 128^2 200 steps")
    _, got, _ = gpu_run(adw, p)
    _, ref, _ = oracle_lib.run_problem(p)
    assert rel_l2(got, ref) <= TOL_RUN["f64"]
    lam = 4 * math.sin(math.pi * p.h / 2) ** 2 / p.h ** 2
    beta = p.dt ** 2 / 2
    g = p.dt ** 2 * 2 * lam / (1 + beta * lam) ** 2
    theta = math.acos(1 - g / 2)
    assert rel_l2(got, math.cos((p.nsteps + 1) * theta) * wl.sine_mode(p.nx, p.ny)) <= TOL_RUN["f64"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c1_paper_start(adw, oracle_lib, dtype):
    p = wl.config_c1(dtype=dtype, nsteps=50, start_mode="paper")
    say(f"C1 paper start {dtype}")
    _, got, _ = gpu_run(adw, p)
    _, ref, _ = oracle_lib.run_problem(p)
    assert rel_l2(got, ref) <= TOL_RUN[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c2_gaussian_pulse_cut(adw, oracle_lib, dtype):
    """C2 shape (2048^2, c = 1, Gaussian pulse, dt = h/2), cut to 200 steps."""
    p = wl.config_c2(dtype=dtype, nsteps=200)
    say(f"C2 {dtype} 2048^2 200 steps")
    _, got, _ = gpu_run(adw, p)
    _, ref, _ = oracle_lib.run_problem(p)
    assert rel_l2(got, ref) <= TOL_RUN[dtype]


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_c2_gaussian_pulse_full(adw, oracle_lib, dtype):
    """C2 in full: 2048^2, 1000 steps."""
    p = wl.config_c2(dtype=dtype)
    say(f"C2 {dtype} 2048^2 1000 steps")
    _, got, _ = gpu_run(adw, p)
    _, ref, _ = oracle_lib.run_problem(p)
    assert rel_l2(got, ref) <= TOL_RUN[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("variant", ["ricker", "pulse"])
def test_c3_shape_at_1024(adw, oracle_lib, dtype, variant):
    """C3's recipe (speed in [1, 3], dt = 0.4 h / max c) at 1024^2 for 300 steps."""
    mk = wl.config_c3 if variant == "ricker" else wl.config_c3p
    p = mk(dtype=dtype, nsteps=300, n=1024)
    say(f"C3-shape {variant} {dtype} 1024^2 300 steps")
    _, got, _ = gpu_run(adw, p)
    _, ref, _ = oracle_lib.run_problem(p)
    assert np.linalg.norm(ref) > 0
    assert rel_l2(got, ref) <= TOL_RUN[dtype]


@pytest.fixture(scope="module")
def c3p_reference(oracle_lib):
    refs = {}

    def get(dtype):
        if dtype not in refs:
            p = wl.config_c3p(dtype=dtype, nsteps=3)
            _, ref, _ = oracle_lib.run_problem(p)
            refs[dtype] = (p, ref)
        return refs[dtype]
    return get


@pytest.mark.parametrize("dtype,one_pass", [("f32", True), ("f32", False), ("f64", False)])
def test_c3_full_size_steps(adw, c3p_reference, dtype, one_pass):
    """C3's grid at its full size (8192^2): 3 steps from a Gaussian pulse over the whole
    field against the oracle, in FP32 with the benchmark's default (one-pass) step and
    with the exact two-pass step, and in FP64 (the paper's arithmetic, exact step):
    relative L2 and the max-norm error relative to max|u|."""
    p, ref = c3p_reference(dtype)
    say(f"C3p {dtype} 8192^2 3 steps one_pass={one_pass}")
    _, got, _ = gpu_run(adw, p, fused_step=one_pass if dtype == "f32" else None)
    e2, em = rel_l2(got, ref), max_rel(got, ref)
    say(f"  rel L2 {e2:.3e}, max-norm {em:.3e}")
    assert e2 <= TOL_RUN[dtype]
    assert em <= TOL_RUN[dtype]


# ------------------------------------------------ starts, sources, traces ----
@pytest.mark.parametrize("mode", ["paper", "ghost"])
def test_start_with_velocity_and_source(adw, oracle_lib, mode):
    n = 77
    h = wl.grid_h(n)
    dt = 0.6 * h
    rng = np.random.default_rng(2)
    c = wl.smooth_field(n, n, 1.0, 2.0, seed=9)
    u0 = wl.gaussian_pulse(n, n, sigma=0.1)
    psi = rng.standard_normal((n, n))
    si = np.array([10 * n + 20, 40 * n + 3], np.int32)
    amp0 = np.array([[3.0, -2.0]])
    say(f"start {mode}")
    wave = adw.Wave(n, n, h, dt, c=dev(c), dtype=torch.float64)
    u1 = wave.start(dev(u0), psi=dev(psi), src_idx=dev(si), src_amp0=dev(amp0), mode=mode)
    torch.cuda.synchronize()
    ref = oracle_lib.start(c * c, u0, h, dt, psi=psi, mode=mode, src_idx=si, src_amp0=amp0)
    assert rel_l2(u1.cpu().numpy(), ref) <= TOL_ONE["f64"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c5_shape_receivers(adw, oracle_lib, dtype):
    """C5's recipe (kappa in [1, 9], Ricker, 64 receivers) at 256^2 for 400 steps."""
    p, _ = wl.config_c5(dtype=dtype, nsteps=400, n=256)
    say(f"C5-shape {dtype} receivers")
    _, got, tr = gpu_run(adw, p, rec=True)
    _, ref, tref = oracle_lib.run_problem(p)
    assert rel_l2(got, ref) <= TOL_RUN[dtype]
    assert np.abs(tref).max() > 0
    assert rel_l2(tr, tref) <= TOL_RUN[dtype]


def test_step_rotation_and_determinism(adw):
    """nsteps in one call equals one-step calls (bitwise); repeated runs are bitwise equal."""
    p = wl.config_c3p(dtype="f32", nsteps=7, n=300)
    say("rotation/determinism")
    wave = adw.Wave(p.nx, p.ny, p.h, p.dt, c=dev(p.c), dtype=torch.float32)
    u0 = dev(p.u0)
    u1 = wave.start(u0)
    a, b = wave.step(u0.clone(), u1.clone(), 7)
    c_, d_ = u0.clone(), u1.clone()
    for _ in range(7):
        c_, d_ = wave.step(c_, d_, 1)
    e, f = wave.step(u0.clone(), u1.clone(), 7)
    torch.cuda.synchronize()
    assert torch.equal(a, c_) and torch.equal(b, d_)
    assert torch.equal(b, f) and torch.equal(a, e)
    # zero steps: nothing changes
    g, h_ = u0.clone(), u1.clone()
    g2, h2 = wave.step(g, h_, 0)
    assert g2 is g and h2 is h_ and torch.equal(h2, u1)


@pytest.mark.parametrize("path", ["one_pass", "two_pass", "one_pass_f64", "two_pass_f64", "cyclic_reduction"])
def test_receiver_traces_every_path(adw, path):
    """Traces of a multi-step call equal those of one-step calls bit for bit, and equal
    each level sampled on the host.  Within a call, a step's receivers are recorded by
    the next step's first launch, and the last step's by a launch of its own.  The test
    uses 1500 receivers (more than one workgroup's threads), with repeated nodes and
    offsets outside the grid, which record NaN."""
    nx, ny, nsteps = 512, 300, 6
    f64 = path.endswith("_f64")
    dt_ = torch.float64 if f64 else torch.float32
    h = 1.0 / (max(nx, ny) + 1)
    c = wl.smooth_field(nx, ny, 1.0, 3.0, seed=8).astype(np.float64 if f64 else np.float32)
    u0 = wl.gaussian_pulse(nx, ny, sigma=0.08).astype(c.dtype)
    rng = np.random.default_rng(8)
    ri = rng.integers(0, nx * ny, 1500).astype(np.int32)
    ri[::97] = ri[1]
    ri[5], ri[700], ri[1499] = -3, nx * ny, nx * ny + 11
    valid = (ri >= 0) & (ri < nx * ny)
    src = np.array([(ny // 2) * nx + nx // 2], np.int32)
    amp = (rng.standard_normal((nsteps, 1)) * 30.0).astype(c.dtype)
    say(f"receiver traces {path}")
    wave = adw.Wave(nx, ny, h, 0.4 * h / 3.0, c=dev(c), dtype=dt_)
    wave.set_tuning(fused_step=path.startswith("one_pass"),
                    cyclic_reduction=True if path == "cyclic_reduction" else None)
    assert wave.info()["fused_step"] == int(path.startswith("one_pass"))
    assert wave.info()["line_solver"] == (2 if path == "cyclic_reduction" else 1)
    a0 = dev(u0)
    b0 = wave.start(a0)
    ridx = dev(ri)
    tr_all = torch.zeros((nsteps, ri.size), dtype=dt_, device="cuda")
    a, b = wave.step(a0.clone(), b0.clone(), nsteps, src_idx=dev(src), src_amp=dev(amp), rec_idx=ridx,
                     traces=tr_all)
    tr_one = torch.zeros_like(tr_all)
    c_, d_ = a0.clone(), b0.clone()
    levels = []
    for k in range(nsteps):
        c_, d_ = wave.step(c_, d_, 1, src_idx=dev(src), src_amp=dev(amp[k:k + 1]), rec_idx=ridx,
                           traces=tr_one[k])
        levels.append(d_.clone())
    torch.cuda.synchronize()
    wave.close()
    assert torch.equal(b, d_)
    ta, to = tr_all.cpu().numpy(), tr_one.cpu().numpy()
    assert np.isnan(ta[:, ~valid]).all() and np.isnan(to[:, ~valid]).all()
    assert np.array_equal(ta[:, valid], to[:, valid])
    for k in range(nsteps):
        assert np.array_equal(ta[k, valid], levels[k].cpu().numpy().ravel()[ri[valid]])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("tr,rs,fused,m", [(64, 3, False, 16), (64, 1, True, 32), (256, 2, False, 32),
                                           (256, 5, True, 16), (1024, 32, False, 32),
                                           (1024, 7, True, 16), (1024, 1, False, 16),
                                           (1024, 1, True, 32)])
def test_launch_plans(adw, oracle_lib, dtype, tr, rs, fused, m):
    """Every admissible launch plan reaches the same answer (10 steps, 300 x 211); the
    one plan that does not fit (the fused FP64 state at 1024 threads per line) is
    rejected before anything runs."""
    nx, ny = 300, 211
    h = 1.0 / 301
    dt = 0.5 * h
    c = wl.smooth_field(nx, ny, 1.0, 3.0, seed=21).astype(npdt(dtype))
    u0 = wl.gaussian_pulse(nx, ny, sigma=0.1).astype(npdt(dtype))
    say(f"plan {dtype} tr={tr} rs={rs} fused={fused} m={m}")
    wave = adw.Wave(nx, ny, h, dt, c=dev(c), dtype=tdt(dtype))
    if fused and dtype == "f64" and tr == 1024:
        before = wave.info()
        with pytest.raises(RuntimeError):
            wave.set_tuning(tr, rs, fused, m, fused_step=False)
        assert wave.info() == before                    # the plan is left as it was
        wave.close()
        return
    wave.set_tuning(tr, rs, fused, m, fused_step=False)
    inf = wave.info()
    assert (inf["x_threads_per_line"], inf["y_fused"], inf["y_chunk_rows"]) == (tr, int(fused), m)
    assert inf["x_rows_per_strip"] == ((32 if m == 16 else 32) if fused else rs)
    assert inf["kernels_per_step"] == (3 if fused else 4)
    a = dev(u0)
    b = wave.start(a)
    a, b = wave.step(a, b, 10)
    torch.cuda.synchronize()
    kap = c.astype(np.float64) ** 2
    u1 = oracle_lib.start(kap, u0, h, dt)
    _, ref, _ = oracle_lib.run(kap, u0, u1, h, dt, 10)
    assert rel_l2(b.cpu().numpy(), ref) <= TOL_RUN[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m", [16, 32])
def test_long_columns(adw, oracle_lib, dtype, m):
    """Columns of 1100 rows: 69 chunks of 16 rows, or 35 of 32, with the y-chunk
    elimination in its own launch (unfused plan); the interface systems take the
    partition solver with 64 threads per column.  Matches the oracle after 10 steps of
    the exact step."""
    nx, ny = 72, 1100
    h = 1.0 / 1101
    dt = 0.5 * h
    c = wl.smooth_field(nx, ny, 1.0, 3.0, seed=23).astype(npdt(dtype))
    u0 = wl.gaussian_pulse(nx, ny, sigma=0.1).astype(npdt(dtype))
    say(f"long columns {dtype} m={m}")
    wave = adw.Wave(nx, ny, h, dt, c=dev(c), dtype=tdt(dtype))
    wave.set_tuning(64, 2, False, m, fused_step=False)
    assert wave.info()["kernels_per_step"] == 4
    a = dev(u0)
    b = wave.start(a)
    a, b = wave.step(a, b, 10)
    torch.cuda.synchronize()
    kap = c.astype(np.float64) ** 2
    u1 = oracle_lib.start(kap, u0, h, dt)
    _, ref, _ = oracle_lib.run(kap, u0, u1, h, dt, 10)
    assert rel_l2(b.cpu().numpy(), ref) <= TOL_RUN[dtype]
    wave.close()


def test_invalid_calls_raise(adw):
    wave = adw.Wave(16, 16, 1 / 17, 0.5 / 17, dtype=torch.float32)
    u = torch.zeros((16, 16), device="cuda")
    with pytest.raises(adw.AdiError):
        wave.step(u, u, 1)                    # same buffer twice
    with pytest.raises(ValueError):
        wave.step(u, torch.zeros((16, 15), device="cuda"), 1)
    with pytest.raises(TypeError):
        wave.step(u, torch.zeros((16, 16), device="cuda", dtype=torch.float64), 1)
    with pytest.raises(adw.AdiError):
        wave.set_tuning(64, 2, False, 24)     # chunk rows must be 16 or 32
    with pytest.raises(adw.AdiError):
        wave.start(u, mode="paper", out=u)    # u1 aliases u0


def test_stream_copy(adw):
    x = torch.randn(1 << 20, device="cuda")
    y = torch.empty_like(x)
    adw.stream_copy(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
