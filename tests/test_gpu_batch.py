"""Batched simulations (many uneven grids in one launch per kernel) against the
FP64 oracle, and the graph / persistent-grid / autotuned plans against the
direct plan (bitwise: they change scheduling only)."""
import numpy as np
import pytest

from tests.conftest import max_rel, rel_l2
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


def tdt(d):
    return torch.float32 if d == "f32" else torch.float64


def npdt(d):
    return np.float32 if d == "f32" else np.float64


def say(msg):
    print(msg, flush=True)


SIZES = [(64, 64), (100, 37), (1, 9), (9, 1), (256, 256), (300, 211), (1000, 50), (33, 517)]


def make_batch(dtype, sizes=SIZES, seed=0):
    sims = []
    for s, (nx, ny) in enumerate(sizes):
        h = 1.0 / (max(nx, ny) + 1)
        c = wl.smooth_field(nx, ny, 1.0, 3.0, seed=100 + s + seed).astype(npdt(dtype))
        dt = 0.45 * h / float(c.max())
        u0 = wl.gaussian_pulse(nx, ny, sigma=0.1).astype(npdt(dtype))
        sims.append(dict(nx=nx, ny=ny, h=h, dt=dt, c=c, u0=u0))
    return sims


def run_batch(adw, sims, dtype, nsteps, graph=False, plan=None, autotune=False):
    t = tdt(dtype)
    b = adw.Batch([(s["nx"], s["ny"]) for s in sims], [s["h"] for s in sims],
                  [s["dt"] for s in sims], [torch.from_numpy(s["c"]).cuda() for s in sims], dtype=t)
    if plan:
        b.set_plan(**plan)
    if autotune:
        b.autotune(trial_steps=3)
    u0 = [torch.from_numpy(s["u0"]).cuda() for s in sims]
    u1 = [torch.zeros_like(x) for x in u0]
    b.bind(u0, u1)
    b.start("ghost")
    if graph:
        b.graph(True)
    b.step(nsteps)
    prev, curr = b.levels()
    torch.cuda.synchronize()
    out = [x.cpu().numpy() for x in curr]
    info = b.plan()
    b.close()
    return out, info


def oracle_run(oracle_lib, s, nsteps):
    kap = s["c"].astype(np.float64) ** 2
    u1 = oracle_lib.start(kap, s["u0"], s["h"], s["dt"])
    _, ref, _ = oracle_lib.run(kap, s["u0"], u1, s["h"], s["dt"], nsteps)
    return ref


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_matches_oracle(adw, oracle_lib, dtype):
    sims = make_batch(dtype)
    say(f"batch {dtype} {len(sims)} sims, 25 steps")
    got, info = run_batch(adw, sims, dtype, 25)
    assert info["count"] == len(sims)
    assert info["fused_allowed"] == 0 and info["fused_step"] == 0   # rows of 1, 9, 33 values
    for s, g in zip(sims, got):
        assert rel_l2(g, oracle_run(oracle_lib, s, 25)) <= TOL[dtype], (s["nx"], s["ny"])


# every row length a multiple of 4: the FP32 batch then runs the one-pass step
SIZES4 = [(64, 64), (100, 37), (4, 9), (8, 1), (256, 256), (300, 211), (1000, 50), (36, 517)]


@pytest.mark.parametrize("lane", [8, 4])
def test_batch_one_pass_matches_oracle(adw, oracle_lib, lane):
    sims = make_batch("f32", sizes=SIZES4, seed=5)
    say(f"batch one-pass f32, {lane} nodes per lane, 25 steps")
    got, info = run_batch(adw, sims, "f32", 25, plan=dict(fused_lane_nodes=lane))
    assert info["fused_allowed"] == 1 and info["fused_step"] == 1 and info["fused_items"] > len(sims)
    assert info["fused_lane_nodes"] == lane
    for s, g in zip(sims, got):
        assert rel_l2(g, oracle_run(oracle_lib, s, 25)) <= TOL["f32"], (s["nx"], s["ny"])


@pytest.mark.parametrize("lane", [8, 4, "strips"])
def test_batch_one_pass_graph_and_exact_step(adw, lane):
    sims = make_batch("f32", sizes=SIZES4, seed=6)
    say(f"batch one-pass graph / exact, {lane} (nodes per lane)")
    plan = dict(fused_strips=True) if lane == "strips" else dict(fused_lane_nodes=lane)
    eager, _ = run_batch(adw, sims, "f32", 11, plan=plan)
    graph, info = run_batch(adw, sims, "f32", 11, graph=True, plan=plan)
    assert info["graph"] == 1 and info["fused_strips"] == (lane == "strips")
    exact, info2 = run_batch(adw, sims, "f32", 11, plan=dict(fused_step=False))
    assert info2["fused_step"] == 0
    for a, b, c in zip(eager, graph, exact):
        assert np.array_equal(a, b)
        assert rel_l2(a, c) <= 3e-6


def strip_plan(nx, ny):
    """a batched simulation's one-pass column strips: the fewest of at most 240
    columns, of one width (a multiple of 8), in segments of at most 1024 rows"""
    tx = -(-nx // 240)
    wt = min(240, (-(-nx // tx) + 7) // 8 * 8)
    seg = -(-ny // 1024)
    hs = -(-ny // seg)
    return wt, hs, -(-nx // wt) * -(-ny // hs)


def plain_strips(adw, p, u0, u1, nsteps, wt, hs):
    """the plain solver on the given column strips"""
    w = adw.Wave(p["nx"], p["ny"], p["h"], p["dt"], c=torch.from_numpy(p["c"]).cuda(), dtype=torch.float32)
    w.set_tuning(fused_step=True, fused_lane_nodes=4, fused_tile_cols=wt, fused_segment_rows=max(hs, 8))
    i = w.info()
    assert (i["fused_step"], i["fused_tile_cols"], i["fused_segment_rows"]) == (1, wt, max(hs, 8))
    _, c = w.step(u0.clone(), u1.clone(), nsteps)
    torch.cuda.synchronize()
    w.close()
    return c.cpu().numpy()


# row lengths a multiple of 4, one to four strips, one or two segments (1100 rows)
SIZES_STRIPS = [(64, 64), (100, 37), (4, 9), (8, 1), (256, 256), (300, 211), (488, 96),
                (1000, 50), (36, 517), (1024, 1100)]


def test_batch_one_pass_strips_match_plain_and_oracle(adw, oracle_lib):
    """The batch's column strips run each simulation exactly as the plain solver on
    the same strips (bitwise), and match the oracle to the FP32 bars."""
    nsteps = 21
    sims = make_batch("f32", sizes=SIZES_STRIPS, seed=8)
    say(f"batch one-pass strips, {len(sims)} sims, {nsteps} steps")
    u0s, u1s = [], []
    for p in sims:
        w = adw.Wave(p["nx"], p["ny"], p["h"], p["dt"], c=torch.from_numpy(p["c"]).cuda(), dtype=torch.float32)
        u0 = torch.from_numpy(p["u0"]).cuda()
        u1s.append(w.start(u0, mode="ghost"))
        u0s.append(u0)
        w.close()
    b = adw.Batch([(p["nx"], p["ny"]) for p in sims], [p["h"] for p in sims], [p["dt"] for p in sims],
                  [torch.from_numpy(p["c"]).cuda() for p in sims], dtype=torch.float32)
    b.set_plan(fused_strips=True)
    b.bind([x.clone() for x in u0s], [x.clone() for x in u1s])
    b.step(nsteps)
    _, curr = b.levels()
    torch.cuda.synchronize()
    info = b.plan()
    got = [x.cpu().numpy() for x in curr]
    b.close()
    assert info["fused_step"] == 1 and info["fused_strips"] == 1
    assert info["fused_items"] == sum(strip_plan(p["nx"], p["ny"])[2] for p in sims)
    for k, p in enumerate(sims):
        wt, hs, _ = strip_plan(p["nx"], p["ny"])
        ref = plain_strips(adw, p, u0s[k], u1s[k], nsteps, wt, hs)
        assert np.array_equal(ref, got[k]), (p["nx"], p["ny"], wt, hs)
        e2, em = rel_l2(got[k], oracle_run(oracle_lib, p, nsteps)), max_rel(got[k], oracle_run(oracle_lib, p, nsteps))
        say(f"  {p['nx']}x{p['ny']} strips {wt} x {hs}: rel L2 {e2:.3e}, max-norm {em:.3e}")
        assert e2 <= TOL["f32"] and em <= TOL["f32"], (p["nx"], p["ny"], e2, em)


def test_batch_plan_strips_round_trip(adw):
    sims = make_batch("f32", sizes=SIZES4[:3])
    b = adw.Batch([(s["nx"], s["ny"]) for s in sims], [s["h"] for s in sims],
                  [s["dt"] for s in sims], [torch.from_numpy(s["c"]).cuda() for s in sims], dtype=torch.float32)
    assert b.plan()["fused_strips"] == 0
    b.set_plan(fused_strips=True, fused_lane_nodes=8)
    p = b.plan()
    assert (p["fused_strips"], p["fused_lane_nodes"]) == (1, 8)
    assert p["fused_items"] == sum(strip_plan(s["nx"], s["ny"])[2] for s in sims)
    b.set_plan(fused_lane_nodes=4)                  # the tile kind only: strips kept
    assert (b.plan()["fused_strips"], b.plan()["fused_lane_nodes"]) == (1, 4)
    b.set_plan(fused_strips=False)
    assert b.plan()["fused_strips"] == 0 and b.plan()["fused_lane_nodes"] == 4
    p = adw._lib.AdiBatchPlan()
    adw._lib.check(adw._lib.load().adi_batch_get_plan(b._h, adw._lib.ctypes.byref(p)))
    p.fused_strips = 3
    assert adw._lib.load().adi_batch_set_plan(b._h, adw._lib.ctypes.byref(p)) != 0
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_graph_and_grids_are_bitwise_equal(adw, dtype):
    sims = make_batch(dtype, seed=7)
    say(f"batch graph/grids {dtype}")
    base, _ = run_batch(adw, sims, dtype, 9)
    with_graph, info = run_batch(adw, sims, dtype, 9, graph=True)
    assert info["graph"] == 1
    persistent, _ = run_batch(adw, sims, dtype, 9, plan=dict(x_grid=5, yscan_grid=3, ysolve_grid=11))
    for a, b, c in zip(base, with_graph, persistent):
        assert np.array_equal(a, b)
        assert np.array_equal(a, c)


def test_batch_autotune_keeps_results(adw, oracle_lib):
    sims = make_batch("f64", sizes=[(128, 96), (511, 64), (77, 300)], seed=3)
    say("batch autotune")
    got, info = run_batch(adw, sims, "f64", 12, autotune=True, graph=True)
    for s, g in zip(sims, got):
        assert rel_l2(g, oracle_run(oracle_lib, s, 12)) <= TOL["f64"]


def test_batch_c4_sample(adw, oracle_lib):
    """Eight simulations drawn by C4's recipe (N in 256..1024, FP32), 40 steps, graph replay."""
    probs = wl.config_c4(dtype="f32", nsteps=40, count=8)
    sims = [dict(nx=p.nx, ny=p.ny, h=p.h, dt=p.dt, c=p.c, u0=p.u0) for p in probs]
    say("batch C4 sample")
    got, _ = run_batch(adw, sims, "f32", 40, graph=True)
    for s, g in zip(sims, got):
        assert rel_l2(g, oracle_run(oracle_lib, s, 40)) <= TOL["f32"]


def widest(nx, wmax):
    """the widest one-pass tiles (the batch's layout): fewest across, multiples of 8"""
    tx = -(-nx // wmax)
    return (-(-nx // tx) + 7) // 8 * 8


def test_batch_c4_full(adw, oracle_lib):
    """C4 at its full size: 256 simulations (N in 256..1024 step 64, FP32), autotuned
    plan, graph replay, 20 steps from levels made by each simulation's own ghost start.
    Every simulation is bitwise equal to the plain solver run on the same tile layout
    (the batch's widest tiles and its nodes per lane), and 8 seeded simulations (with
    the smallest and the largest grid) match the oracle to the FP32 bars."""
    nsteps = 20
    probs = wl.config_c4(dtype="f32", nsteps=nsteps)
    assert len(probs) == 256
    say("batch C4 full: 256 sims, plain ghost starts")
    u0s, u1s = [], []
    for p in probs:
        w = adw.Wave(p.nx, p.ny, p.h, p.dt, c=torch.from_numpy(p.c).cuda(), dtype=torch.float32)
        u0 = torch.from_numpy(p.u0).cuda()
        u1s.append(w.start(u0, mode="ghost"))
        u0s.append(u0)
        w.close()
    torch.cuda.synchronize()
    b = adw.Batch([(p.nx, p.ny) for p in probs], [p.h for p in probs], [p.dt for p in probs],
                  [torch.from_numpy(p.c).cuda() for p in probs], dtype=torch.float32)
    b.autotune(trial_steps=3)
    lv0 = [x.clone() for x in u0s]
    lv1 = [x.clone() for x in u1s]
    b.bind(lv0, lv1)
    b.graph(True)
    b.step(nsteps)
    _, curr = b.levels()
    torch.cuda.synchronize()
    info = b.plan()
    assert info["count"] == 256 and info["graph"] == 1 and info["fused_step"] == 1
    lane, strips = info["fused_lane_nodes"], info["fused_strips"]
    say(f"  autotuned plan: {'column strips' if strips else f'tiles of {lane} nodes per lane'}, "
        f"x threads {info['x_threads_per_line']}")
    got = [x.cpu().numpy() for x in curr]
    b.close()
    say("batch C4 full: plain runs on the same tiles or strips")
    for s, p in enumerate(probs):
        if strips:
            wt, hs, _ = strip_plan(p.nx, p.ny)
            ref = plain_strips(adw, dict(nx=p.nx, ny=p.ny, h=p.h, dt=p.dt, c=p.c), u0s[s], u1s[s], nsteps, wt, hs)
            assert np.array_equal(ref, got[s]), (s, p.nx)
            continue
        w = adw.Wave(p.nx, p.ny, p.h, p.dt, c=torch.from_numpy(p.c).cuda(), dtype=torch.float32)
        w.set_tuning(fused_step=True, fused_lane_nodes=lane, fused_segment_rows=-2,
                     fused_tile_cols=widest(p.nx, 240 if lane == 4 else 496))
        a, c = w.step(u0s[s].clone(), u1s[s].clone(), nsteps)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy(), got[s]), (s, p.nx)
        w.close()
    rng = np.random.default_rng(44)
    sizes = np.array([p.nx for p in probs])
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes))}
    while len(pick) < 8:
        pick.add(int(rng.integers(0, 256)))
    for s in sorted(pick):
        p = probs[s]
        kap = p.c.astype(np.float64) ** 2
        u1 = oracle_lib.start(kap, p.u0, p.h, p.dt)
        _, ref, _ = oracle_lib.run(kap, p.u0, u1, p.h, p.dt, nsteps)
        e2, em = rel_l2(got[s], ref), max_rel(got[s], ref)
        say(f"  sim {s} ({p.nx}^2): rel L2 {e2:.3e}, max-norm {em:.3e}")
        assert e2 <= TOL["f32"] and em <= TOL["f32"], (s, e2, em)


def test_batch_levels_rotate_and_errors(adw):
    sims = make_batch("f32", sizes=[(40, 30), (20, 50)])
    b = adw.Batch([(s["nx"], s["ny"]) for s in sims], [s["h"] for s in sims],
                  [s["dt"] for s in sims], [1.5, 2.0], dtype=torch.float32)
    u0 = [torch.from_numpy(s["u0"]).cuda() for s in sims]
    u1 = [torch.zeros_like(x) for x in u0]
    with pytest.raises(adw.AdiError):
        b.step(1)                                   # not bound yet
    b.bind(u0, u1)
    b.start("paper")
    b.step(3)
    prev, curr = b.levels()
    assert all(c is a for c, a in zip(curr, u0))    # odd count: roles swapped
    b.step(1)
    prev, curr = b.levels()
    assert all(c is a for c, a in zip(curr, u1))
    with pytest.raises(adw.AdiError):
        b.start("ghost")                            # only before the first step
    b.close()
