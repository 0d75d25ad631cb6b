"""Adjoint (reverse-time) gradients on the GPU against the FP64 oracle's adjoint,
finite differences of the GPU forward, the dot-product identity, checkpoint
invariance, the forward-record checks and the autograd Function.

Tolerances (relative L2 against the oracle's adjoint, computed in FP64):
  FP64 gradients <= 1e-12, FP32 gradients <= 1e-5 (the run's bars).
Each FP32 case also reports the drift of a correctly rounded FP32 transcription
of the same recurrences (tests/drift_gauge.py) against the same oracle; the GPU
error is asserted to stay within 4x that inherent drift as well."""
import numpy as np
import pytest

from tests import drift_gauge
from tests.conftest import rel_l2
from paper_2006_10142_amd import workloads as wl

TOL_GRAD = {"f64": 1e-12, "f32": 1e-5}
TOL_TRACE = {"f64": 1e-12, "f32": 1e-5}

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def adw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2006_10142_amd as m
    m._lib.load()
    return m


def tdt(d):
    return torch.float32 if d == "f32" else torch.float64


def npdt(d):
    return np.float32 if d == "f32" else np.float64


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(msg):
    print(msg, flush=True)


def case(dtype, nx=90, ny=70, nsteps=50, seed=1, nonzero=False):
    h = 1.0 / (max(nx, ny) + 1)
    kappa = wl.smooth_field(nx, ny, 1.0, 9.0, seed=seed).astype(npdt(dtype))
    dt = 0.4 * h / 3.0
    rng = np.random.default_rng(seed)
    if nonzero:
        up = (0.1 * wl.gaussian_pulse(nx, ny, 0.1)).astype(npdt(dtype))
        uc = (up.astype(np.float64) * 0.999).astype(npdt(dtype))
    else:
        up = np.zeros((ny, nx), npdt(dtype))
        uc = np.zeros((ny, nx), npdt(dtype))
    src_idx = np.array([(ny // 3) * nx + nx // 2, (2 * ny // 3) * nx + nx // 4], np.int32)
    amp = (wl.point_source_series(nsteps, dt, h, 1, f0=25.0) * np.array([[1.0, -0.5]])).astype(npdt(dtype))
    rec_idx = np.array([(ny // 8) * nx + (k * nx) // 8 for k in range(8)], np.int32)
    target = (rng.standard_normal((nsteps, 8)) * 1e-4).astype(npdt(dtype))
    return dict(nx=nx, ny=ny, h=h, dt=dt, kappa=kappa, up=up, uc=uc, src_idx=src_idx, amp=amp,
                rec_idx=rec_idx, target=target, nsteps=nsteps, dtype=dtype)


def gpu_grad(adw, c, K, want_amp=True, kappa=None, one_pass=None):
    """one_pass: True / False forces the forward run's step (one-pass / exact
    two-pass), None keeps the handle's choice."""
    wave = adw.Wave(c["nx"], c["ny"], c["h"], c["dt"], dtype=tdt(c["dtype"]),
                    kappa=dev(c["kappa"] if kappa is None else kappa))
    if one_pass is not None:
        wave.set_tuning(fused_step=one_pass)
        assert wave.info()["fused_step"] == int(one_pass)
    si, ri = dev(c["src_idx"]), dev(c["rec_idx"])
    amp = dev(c["amp"])
    tr = wave.adjoint_forward(dev(c["up"]), dev(c["uc"]), c["nsteps"], src_idx=si, src_amp=amp,
                              rec_idx=ri, checkpoint_every=K)
    gtr = 2.0 * (tr - dev(c["target"]))
    gk, ga = wave.adjoint_backward(gtr, src_idx=si, src_amp=amp, rec_idx=ri, want_amp=want_amp)
    torch.cuda.synchronize()
    out = (gk.cpu().numpy(), None if ga is None else ga.cpu().numpy(), tr.cpu().numpy())
    wave.close()
    return out


def oracle_grad(oracle_lib, c):
    kap = c["kappa"].astype(np.float64)
    _, _, tr = oracle_lib.run(kap, c["up"], c["uc"], c["h"], c["dt"], c["nsteps"], src_idx=c["src_idx"],
                              src_amp=c["amp"], rec_idx=c["rec_idx"])
    gk, ga = oracle_lib.adjoint(kap, c["up"], c["uc"], c["h"], c["dt"], c["nsteps"],
                                2.0 * (tr - c["target"]), c["rec_idx"], src_idx=c["src_idx"],
                                src_amp=c["amp"])
    return gk, ga, tr


def gauge_grad(c):
    """dJ/dkappa, dJ/dsource of the same case by the float32 transcription."""
    gk, ga, _ = drift_gauge.misfit_gradient(c["kappa"], c["up"], c["uc"], c["h"], c["dt"], c["nsteps"],
                                            c["src_idx"], c["amp"], c["rec_idx"], c["target"],
                                            dtype=np.float32)
    return gk, ga


def check_grads(c, got, ref, what):
    """Assert the bars; FP32 also against 4x the inherent FP32 drift.  The measured
    errors are printed and carried in every assertion message."""
    (gk, ga, tr), (rk, ra, rtr) = got, ref
    dtype = c["dtype"]
    e = dict(traces=rel_l2(tr, rtr), kappa=rel_l2(gk, rk), source=rel_l2(ga, ra))
    msg = f"{what} {dtype}: rel L2 traces {e['traces']:.3e} dJ/dkappa {e['kappa']:.3e} dJ/dsource {e['source']:.3e}"
    if dtype == "f32":
        qk, qa = gauge_grad(c)
        gq = dict(kappa=rel_l2(qk, rk), source=rel_l2(qa, ra))
        msg += f"; FP32 drift of the same recurrence: dJ/dkappa {gq['kappa']:.3e} dJ/dsource {gq['source']:.3e}"
    say("  " + msg)
    assert np.abs(rk).max() > 0, msg
    assert e["traces"] <= TOL_TRACE[dtype], msg
    assert e["kappa"] <= TOL_GRAD[dtype], msg
    assert e["source"] <= TOL_GRAD[dtype], msg
    if dtype == "f32":
        assert e["kappa"] <= 4 * gq["kappa"] and e["source"] <= 4 * gq["source"], msg


@pytest.mark.parametrize("dtype,K,nonzero", [("f64", 1, False), ("f64", 7, True), ("f64", 50, False),
                                             ("f32", 16, False), ("f32", 50, True)])
def test_adjoint_matches_oracle(adw, oracle_lib, dtype, K, nonzero):
    c = case(dtype, nonzero=nonzero)
    say(f"adjoint {dtype} K={K} nonzero={nonzero}")
    check_grads(c, gpu_grad(adw, c, K), oracle_grad(oracle_lib, c), f"K={K} nonzero={nonzero}")


@pytest.mark.parametrize("dtype,K,nonzero", [("f64", 7, True), ("f64", 50, False), ("f32", 16, False),
                                             ("f32", 50, True)])
def test_adjoint_one_pass_forward_matches_oracle(adw, oracle_lib, dtype, K, nonzero):
    """The forward run and the recomputation on the one-pass step (96 x 70, so every
    row length allows it), against the oracle's exact adjoint: the one-pass step
    differs from the exact one by at most half an ulp per step, so the same bars hold."""
    c = case(dtype, nx=96, nonzero=nonzero)
    say(f"adjoint on the one-pass step {dtype} K={K} nonzero={nonzero}")
    check_grads(c, gpu_grad(adw, c, K, one_pass=True), oracle_grad(oracle_lib, c), f"one-pass K={K}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_one_pass_checkpoint_interval(adw, dtype):
    """After a one-pass forward run the reverse pass works on the exact step's
    levels recomputed from the checkpoints, which differ from the forward run's by at
    most the one-pass bound (half an ulp per step): the gradient then depends on the
    checkpoint interval only at that level (FP64 1e-13, FP32 2e-6 relative L2); the
    traces do not depend on it at all."""
    c = case(dtype, nx=96, ny=48, nsteps=37, seed=4)
    say(f"one-pass checkpoint interval {dtype}")
    g = [gpu_grad(adw, c, K, one_pass=True) for K in (1, 5, 37, 100)]
    tol = 1e-13 if dtype == "f64" else 2e-6
    for x in g[1:]:
        assert np.array_equal(g[0][2], x[2])
        e = (rel_l2(x[0], g[0][0]), rel_l2(x[1], g[0][1]))
        say(f"  dJ/dkappa {e[0]:.3e}, dJ/dsource {e[1]:.3e} against K = 1")
        assert e[0] <= tol and e[1] <= tol, e


@pytest.mark.parametrize("nx,ny", [(30, 50), (7, 90), (130, 9), (2100, 12), (2101, 12)])
def test_adjoint_narrow_grids(adw, oracle_lib, nx, ny):
    """Grids narrower than one 64-wide block of the reverse kernels, and wide, short
    ones (rows of more than 2048 nodes take the separate transposed x-solve and update
    kernels, 2101 the update without 16-byte vectors): gradients of kappa and of the
    source values against the oracle (FP64)."""
    c = case("f64", nx=nx, ny=ny, nsteps=24, seed=nx + ny)
    say(f"adjoint narrow {nx}x{ny}")
    got = gpu_grad(adw, c, 5)
    ref = oracle_grad(oracle_lib, c)
    assert np.abs(ref[1]).max() > 0
    check_grads(c, got, ref, f"narrow {nx}x{ny}")


@pytest.mark.parametrize("dtype,one_pass", [("f64", None), ("f32", None), ("f32", True)])
def test_adjoint_long_columns(adw, oracle_lib, dtype, one_pass):
    """Columns of 1100 rows (69 chunks of 16, so the interface systems of the forward
    run, the recomputation and the transposed y-lines take 64 threads per column; on the
    FP32 one-pass step the transposed y-lines run on windows: 35 segments of 32 rows, the
    last one ragged), sources and receivers 10 rows apart in the middle of the grid."""
    c = case(dtype, nx=24, ny=1100, nsteps=24, seed=17)
    nx = c["nx"]
    c["src_idx"] = np.array([550 * nx + 12, 552 * nx + 5], np.int32)
    c["rec_idx"] = np.array([560 * nx + 2 * k + 3 for k in range(8)], np.int32)
    say(f"adjoint long columns {dtype} one-pass {one_pass}")
    got = gpu_grad(adw, c, 5, one_pass=one_pass)
    ref = oracle_grad(oracle_lib, c)
    assert np.abs(ref[1]).max() > 0
    check_grads(c, got, ref, "long columns")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_shared_receiver_nodes(adw, oracle_lib, dtype):
    """300 receivers (more than one 256-wide tile) with repeated nodes, one of them on a
    source node, and one offset outside the grid."""
    c = case(dtype, nx=64, ny=40, nsteps=30, seed=11)
    nx, ny = c["nx"], c["ny"]
    rng = np.random.default_rng(3)
    base = rng.integers(0, nx * ny, size=120).astype(np.int32)
    ri = np.concatenate([base, base[:100], base[:60], base[:19], c["src_idx"][:1]]).astype(np.int32)
    rng.shuffle(ri)
    ri = np.concatenate([ri, np.array([nx * ny + 5], np.int32)])
    assert ri.size == 301
    c["rec_idx"] = ri
    c["target"] = (rng.standard_normal((c["nsteps"], ri.size)) * 1e-4).astype(npdt(dtype))
    say(f"shared receivers {dtype}")
    gk, ga, tr = gpu_grad(adw, c, 7)
    valid = ri < nx * ny
    assert np.isnan(tr[:, ~valid]).all()
    c2 = dict(c, rec_idx=ri[valid], target=c["target"][:, valid])
    check_grads(c2, (gk, ga, tr[:, valid]), oracle_grad(oracle_lib, c2), "shared receivers")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_checkpoint_interval_does_not_change_the_gradient(adw, dtype):
    c = case(dtype, nx=64, ny=48, nsteps=37, seed=4)
    say(f"checkpoint invariance {dtype}")
    g1 = gpu_grad(adw, c, 1)
    g2 = gpu_grad(adw, c, 5)
    g3 = gpu_grad(adw, c, 37)
    g4 = gpu_grad(adw, c, 100)
    for g in (g2, g3, g4):
        assert np.array_equal(g1[0], g[0]) and np.array_equal(g1[1], g[1])


@pytest.mark.parametrize("n,nsteps,nrec", [(128, 300, 16), (1024, 2000, 64)])
def test_gradient_matches_finite_differences_on_gpu(adw, n, nsteps, nrec):
    """C5's recipe (kappa in [1, 9], Ricker, receivers on the row nearest y = 0.1,
    checkpoints every 100 steps), FP64: central differences of the GPU loss, with
    eps = 1e-5 kappa, agree with the adjoint gradient to 1e-5 on 16 cells: the source
    node (where dJ/dkappa peaks, hundreds of times above every other node at C5's full
    size) and 15 seeded cells with |dJ/dkappa| >= 0.3 of the largest value outside the
    source's 5x5 neighbourhood.  Smaller gradients are not FD-checkable at this eps: the
    loss carries about 1e-15 relative rounding after 2000 steps, which the quotient turns
    into about 1e-11 absolute, 1e-5 of a gradient of 1e-6 (measured at C5's full size).
    (1024, 2000, 64) is C5 at its full size."""
    p, kt = wl.config_c5(dtype="f64", nsteps=nsteps, n=n, nrec=nrec)
    # target: the traces of the run on the second kappa field
    wave = adw.Wave(p.nx, p.ny, p.h, p.dt, dtype=torch.float64, kappa=dev(kt))
    si, ri, amp = dev(p.src_idx), dev(p.rec_idx), dev(p.src_amp)
    zero = dev(p.u_prev)
    target = wave.adjoint_forward(zero, zero, p.nsteps, src_idx=si, src_amp=amp, rec_idx=ri,
                                  checkpoint_every=100)
    say(f"C5 FD check {n}^2 {nsteps} steps")

    def loss(kap):
        wave.set_kappa(dev(kap))
        tr = wave.adjoint_forward(zero, zero, p.nsteps, src_idx=si, src_amp=amp, rec_idx=ri,
                                  checkpoint_every=100)
        return float(((tr - target) ** 2).sum()), tr

    J0, tr = loss(p.kappa)
    assert J0 > 0
    gk, _ = wave.adjoint_backward(2.0 * (tr - target), src_idx=si, src_amp=amp, rec_idx=ri)
    g = gk.cpu().numpy()
    rng = np.random.default_rng(6)
    sj, si0 = divmod(int(p.src_idx[0]), p.nx)
    away = np.abs(g).copy()
    away[max(sj - 2, 0):sj + 3, max(si0 - 2, 0):si0 + 3] = 0.0
    cand = np.argwhere(away >= 0.3 * away.max())
    cells = [(sj, si0)] + [tuple(c) for c in cand[rng.choice(len(cand), size=15, replace=False)]]
    worst = 0.0
    for (j, i) in cells:
        eps = 1e-5 * p.kappa[j, i]
        kp = p.kappa.copy(); kp[j, i] += eps
        km = p.kappa.copy(); km[j, i] -= eps
        fd = (loss(kp)[0] - loss(km)[0]) / (2 * eps)
        err = abs(fd - g[j, i]) / abs(fd)
        worst = max(worst, err)
        assert err <= 1e-5, (j, i, fd, g[j, i], err)
    say(f"  FD vs adjoint: worst relative difference over 16 cells {worst:.3e}")
    wave.close()


@pytest.mark.parametrize("full", [False, True])
def test_dot_product_identity_on_gpu(adw, full):
    """<F f, d> = <f, F^T d> for the linear map source values -> traces (FP64, zero start),
    to 1e-13 of |<F f, d>|, with d = F f plus seeded noise of the same size.  full: C5 at
    its full size (1024^2, 2000 steps, 64 receivers, checkpoints every 100 steps)."""
    if full:
        p, _ = wl.config_c5(dtype="f64")
        c = dict(nx=p.nx, ny=p.ny, h=p.h, dt=p.dt, kappa=p.kappa, up=p.u_prev, uc=p.u_curr,
                 src_idx=p.src_idx, amp=p.src_amp, rec_idx=p.rec_idx, nsteps=p.nsteps)
        K = 100
    else:
        c = case("f64", nx=80, ny=60, nsteps=60, seed=8)
        K = 13
    say(f"dot product {'C5 full' if full else '80x60'}")
    wave = adw.Wave(c["nx"], c["ny"], c["h"], c["dt"], dtype=torch.float64, kappa=dev(c["kappa"]))
    si, ri, amp = dev(c["src_idx"]), dev(c["rec_idx"]), dev(c["amp"])
    Ff = wave.adjoint_forward(dev(c["up"]), dev(c["uc"]), c["nsteps"], src_idx=si, src_amp=amp,
                              rec_idx=ri, checkpoint_every=K).cpu().numpy()
    rng = np.random.default_rng(2)
    d = Ff + np.sqrt(np.mean(Ff ** 2)) * rng.standard_normal(Ff.shape)
    _, Ftd = wave.adjoint_backward(dev(d), src_idx=si, src_amp=amp, rec_idx=ri, want_amp=True)
    lhs = float((Ff * d).sum())
    rhs = float((c["amp"] * Ftd.cpu().numpy()).sum())
    rel = abs(lhs - rhs) / abs(lhs)
    norm = abs(lhs - rhs) / (np.linalg.norm(Ff) * np.linalg.norm(d))
    say(f"  |lhs - rhs| / |lhs| = {rel:.3e}, / (|Ff| |d|) = {norm:.3e}")
    assert abs(lhs) > 0
    assert rel <= 1e-13, (lhs, rhs, rel)
    wave.close()


def test_autograd_function(adw, oracle_lib):
    c = case("f64", nx=48, ny=40, nsteps=30, seed=5)
    wave = adw.Wave(c["nx"], c["ny"], c["h"], c["dt"], dtype=torch.float64, kappa=dev(c["kappa"]))
    kap = dev(c["kappa"]).requires_grad_(True)
    amp = dev(c["amp"]).requires_grad_(True)
    si, ri = dev(c["src_idx"]), dev(c["rec_idx"])
    tr = adw.simulate_traces(wave, kap, dev(c["up"]), dev(c["uc"]), c["nsteps"], si, amp, ri,
                             checkpoint_every=8)
    loss = ((tr - dev(c["target"])) ** 2).sum()
    loss.backward()
    rk, ra, _ = oracle_grad(oracle_lib, c)
    assert rel_l2(kap.grad.cpu().numpy(), rk) <= TOL_GRAD["f64"]
    assert rel_l2(amp.grad.cpu().numpy(), ra) <= TOL_GRAD["f64"]
    wave.close()


def test_forward_record_is_checked(adw, oracle_lib):
    """One stored forward run per handle: a backward for a run that a later forward
    replaced, or after a coefficient change, raises instead of returning another run's
    gradient; the latest run's backward stays exact."""
    c = case("f64", nx=40, ny=36, nsteps=20, seed=14)
    wave = adw.Wave(c["nx"], c["ny"], c["h"], c["dt"], dtype=torch.float64, kappa=dev(c["kappa"]))
    si, ri, amp = dev(c["src_idx"]), dev(c["rec_idx"]), dev(c["amp"])
    up, uc = dev(c["up"]), dev(c["uc"])
    tr1 = wave.adjoint_forward(up, uc, c["nsteps"], src_idx=si, src_amp=amp, rec_idx=ri, checkpoint_every=6)
    first = wave.adjoint_record
    amp2 = amp * 0.5
    tr2 = wave.adjoint_forward(up, uc, c["nsteps"], src_idx=si, src_amp=amp2, rec_idx=ri, checkpoint_every=6)
    second = wave.adjoint_record
    assert first != 0 and second != 0 and first != second
    g = 2.0 * (tr1 - dev(c["target"]))
    with pytest.raises(adw.AdiError):
        wave.adjoint_backward(g, src_idx=si, src_amp=amp, rec_idx=ri, record=first)
    # the second run's backward (by id, and by 0 = the stored run) is the oracle's
    c2 = dict(c, amp=c["amp"] * 0.5)
    rk, _, rtr = oracle_grad(oracle_lib, c2)
    assert rel_l2(tr2.cpu().numpy(), rtr) <= TOL_TRACE["f64"]
    for rec_id in (second, 0):
        gk, _ = wave.adjoint_backward(2.0 * (tr2 - dev(c["target"])), src_idx=si, src_amp=amp2, rec_idx=ri,
                                      record=rec_id)
        assert rel_l2(gk.cpu().numpy(), rk) <= TOL_GRAD["f64"]
    # a coefficient change discards the stored run
    wave.set_kappa(dev(c["kappa"]))
    with pytest.raises(adw.AdiError):
        wave.adjoint_backward(g, src_idx=si, src_amp=amp2, rec_idx=ri)
    wave.close()


def test_autograd_two_forwards_before_backward(adw):
    """Two autograd forwards on one handle before the first backward: that backward
    raises (the handle keeps only the second run's checkpoints)."""
    c = case("f64", nx=32, ny=30, nsteps=12, seed=15)
    wave = adw.Wave(c["nx"], c["ny"], c["h"], c["dt"], dtype=torch.float64, kappa=dev(c["kappa"]))
    si, ri = dev(c["src_idx"]), dev(c["rec_idx"])
    kap = dev(c["kappa"]).requires_grad_(True)
    amp = dev(c["amp"])
    tr1 = adw.simulate_traces(wave, kap, dev(c["up"]), dev(c["uc"]), c["nsteps"], si, amp, ri, checkpoint_every=5)
    tr2 = adw.simulate_traces(wave, kap, dev(c["up"]), dev(c["uc"]), c["nsteps"], si, amp * 2, ri,
                              checkpoint_every=5)
    with pytest.raises(adw.AdiError):
        (tr1 ** 2).sum().backward()
    (tr2 ** 2).sum().backward()           # the stored run's backward works
    assert torch.isfinite(kap.grad).all() and float(kap.grad.abs().max()) > 0
    wave.close()
