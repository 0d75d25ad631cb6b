"""The one-pass FP32 step (truncated line solves on overlapping tiles and on column
strips): its plan selection and truncation-bound switch, parity with the FP64 oracle (the exact
two-pass scheme) over tile and strip layouts with ragged edges, point sources and receivers,
and agreement with the GPU's exact two-pass step.

The truncation error of one step is kept below 2^-24 of max|w| by the plan (it
runs only when r <= 0.18 everywhere), so the FP32 bar of the exact path applies:
relative L2 <= 1e-5 against the oracle after the run, and, since that bound is a
max-norm statement, the max-norm error relative to max|u| <= 1e-5 as well."""
import numpy as np
import pytest

from tests.conftest import max_rel, rel_l2
from paper_2006_10142_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL_MAX = 1e-5


def check(got, ref, tol=TOL, tol_max=TOL_MAX, what=""):
    """relative L2 and max-norm error (relative to max|ref|), both asserted"""
    e2, em = rel_l2(got, ref), max_rel(got, ref)
    msg = f"{what}: rel L2 {e2:.3e}, max-norm {em:.3e}"
    say("  " + msg)
    assert e2 <= tol, msg
    assert em <= tol_max, msg


@pytest.fixture(scope="module")
def adw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2006_10142_amd as m
    m._lib.load()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(msg):
    print(msg, flush=True)


def case(nx, ny, cfl=0.4, seed=3, nsteps=30, nsrc=2, nrec=6, f64=False):
    npd = np.float64 if f64 else np.float32
    h = 1.0 / (max(nx, ny) + 1)
    c = wl.smooth_field(nx, ny, 1.0, 3.0, seed=seed).astype(npd)
    dt = cfl * h / 3.0
    u0 = wl.gaussian_pulse(nx, ny, sigma=0.08).astype(npd)
    rng = np.random.default_rng(seed)
    si = np.stack([rng.integers(0, ny, nsrc), rng.integers(0, nx, nsrc)], 1)
    src_idx = (si[:, 0] * nx + si[:, 1]).astype(np.int32)
    amp = (rng.standard_normal((nsteps, nsrc)) * 50.0).astype(npd)
    ri = np.stack([rng.integers(0, ny, nrec), rng.integers(0, nx, nrec)], 1)
    rec_idx = (ri[:, 0] * nx + ri[:, 1]).astype(np.int32)
    return dict(nx=nx, ny=ny, h=h, dt=dt, c=c, u0=u0, src_idx=src_idx, amp=amp, rec_idx=rec_idx,
                nsteps=nsteps, dtype=torch.float64 if f64 else torch.float32)


def gpu(adw, k, one_pass):
    wave = adw.Wave(k["nx"], k["ny"], k["h"], k["dt"], c=dev(k["c"]), dtype=k["dtype"])
    wave.set_tuning(fused_step=one_pass, fused_lane_nodes=k.get("lane", 0), fused_tile_cols=k.get("tile_cols", 0),
                    fused_segment_rows=k.get("hs", 0))
    info = wave.info()
    assert info["fused_step"] == int(one_pass)
    a = dev(k["u0"])
    b = wave.start(a)
    tr = torch.zeros((k["nsteps"], k["rec_idx"].size), dtype=k["dtype"], device="cuda")
    a, b = wave.step(a, b, k["nsteps"], src_idx=dev(k["src_idx"]), src_amp=dev(k["amp"]),
                     rec_idx=dev(k["rec_idx"]), traces=tr)
    torch.cuda.synchronize()
    out = (b.cpu().numpy(), tr.cpu().numpy(), info)
    wave.close()
    return out


def oracle(oracle_lib, k):
    kap = k["c"].astype(np.float64) ** 2
    u1 = oracle_lib.start(kap, k["u0"], k["h"], k["dt"])
    _, ref, tr = oracle_lib.run(kap, k["u0"], u1, k["h"], k["dt"], k["nsteps"], src_idx=k["src_idx"],
                                src_amp=k["amp"], rec_idx=k["rec_idx"])
    return ref, tr


def test_plan_selection_and_bound(adw):
    def info(nx, ny, dt_over_h, dtype=torch.float32, c=1.0):
        w = adw.Wave(nx, ny, 1.0 / (max(nx, ny) + 1), dt_over_h / (max(nx, ny) + 1), c=c, dtype=dtype)
        i = w.info()
        w.close()
        return i
    i = info(2048, 2048, 0.5)                       # C2: r = 1/8
    assert abs(i["r_max"] - 0.125) < 1e-6
    assert i["fused_allowed"] == 1 and i["fused_step"] == 1 and i["kernels_per_step"] == 1
    # FP64: the bound 4 qs^17 <= 2^-53 of the FP64 column strips (K = 16)
    i = info(2048, 2048, 0.5, dtype=torch.float64)                # r = 0.125, qs = 0.101
    assert abs(i["r_max"] - 0.125) < 1e-12
    assert i["fused_allowed"] == 1 and i["fused_step"] == 1 and i["fused_segment_rows"] > 0
    assert info(1024, 1024, 0.51, dtype=torch.float64)["fused_allowed"] == 1   # r = 0.130
    assert info(1024, 1024, 0.52, dtype=torch.float64)["fused_allowed"] == 0   # r = 0.135: bound fails
    assert info(1023, 1024, 0.5, dtype=torch.float64)["fused_allowed"] == 0    # rows not 16-byte multiples
    assert info(128, 128, 0.5, dtype=torch.float64)["fused_step"] == 0         # small grids keep two passes
    assert info(1022, 1024, 0.5)["fused_allowed"] == 0            # rows not 16-byte multiples
    assert info(1024, 1024, 0.58)["fused_allowed"] == 1           # r = 0.168
    assert info(1024, 1024, 0.62)["fused_allowed"] == 0           # r = 0.192: bound fails
    assert info(128, 128, 0.5)["fused_step"] == 0                 # small grids keep two passes
    w = adw.Wave(1024, 1024, 1.0 / 1025, 0.62 / 1025, c=1.0, dtype=torch.float32)
    with pytest.raises(RuntimeError):
        w.set_tuning(fused_step=True)
    w.close()


def widest(nx, wmax=496):
    """the widest tile layout: fewest tiles across, each a multiple of 8 columns"""
    tx = -(-nx // wmax)
    return (-(-nx // tx) + 7) // 8 * 8


def plan(nx, ny, ncu, wmax, ta, tb):
    """the plan's width for one lane variant: least rounds * (ta + tb * width)"""
    best, cost = None, None
    tx0 = -(-nx // wmax)
    tx = tx0
    while tx <= -(-nx // 64):
        wt = (-(-nx // tx) + 7) // 8 * 8
        if wt < 64 and tx > tx0:
            break
        tiles = -(-nx // wt) * -(-ny // 64)
        c = -(-tiles // ncu) * (ta + tb * wt)
        if cost is None or c < cost:
            best, cost = wt, c
        tx += 1
    return best, cost


def balanced(nx, ny, ncu):
    """(nodes per lane, width) of the tile plan: the cheaper of the two variants"""
    w8, c8 = plan(nx, ny, ncu, 496, 16000, 30)
    w4, c4 = plan(nx, ny, ncu, 240, 12000, 15)
    return (4, w4) if c4 < c8 else (8, w8)


def strip_plan(nx, ny, ncu):
    """Column strips as the plan picks them: for tx strips from the fewest of at most
    240 columns, widths w0 and w0 + 8 (a strips of w0 + 8) covering nx, g = ncu // tx
    segments of h rows; the least (widest + 16) * h among those with h >= 256.
    Returns (widest, tx, a or tx, h) or None."""
    best = None
    tx0 = -(-nx // 240)
    for tx in range(tx0, tx0 + 5):
        w0 = nx // tx // 8 * 8
        a = -(-(nx - tx * w0) // 8)
        wmax = w0 + 8 if a > 0 else w0
        g = ncu // tx
        if w0 < 8 or wmax > 240 or a > tx or g <= 0:
            continue
        h = -(-ny // g)
        if h < 256:
            continue
        cost = (wmax + 16) * h
        if best is None or cost < best[0]:
            best = (cost, (wmax, tx, a if a > 0 else tx, h))
    return best[1] if best else None


def auto_plan(nx, ny, ncu):
    """(nodes per lane, width, strip segment rows or 0) the plan picks: column strips
    (strip_plan) when every segment gets at least 256 rows, else the tile plan"""
    sp = strip_plan(nx, ny, ncu)
    if sp:
        return 4, sp[0], sp[3]
    return balanced(nx, ny, ncu) + (0,)


STRIP_LAYOUTS = {"strips_h8": 8, "strips_h30": 30, "strips_h1000": 1000}


@pytest.mark.parametrize("nx,ny", [(480, 64), (488, 65), (1000, 700), (960, 130), (64, 64), (2048, 300),
                                   (4, 200), (1504, 33), (64, 1), (40, 3)])
@pytest.mark.parametrize("layout", ["auto", "lane8", "lane8_widest", "lane4", "lane4_widest"] + sorted(STRIP_LAYOUTS))
def test_one_pass_matches_oracle(adw, oracle_lib, nx, ny, layout):
    """layouts: the automatic plan; eight or four nodes per lane (four: r kept in LDS
    for the y-lines), each on the plan's width and on the widest tiles; column strips
    with 8, 30 and 1000 output rows per segment (bands cut anywhere, segments shorter
    than a band, a strip longer than the grid)"""
    k = case(nx, ny, seed=nx + ny)
    strips = layout in STRIP_LAYOUTS
    k["lane"] = {"auto": -1, "lane8": 8, "lane8_widest": 8, "lane4": 4, "lane4_widest": 4}.get(layout, 0)
    k["tile_cols"] = widest(nx, 240 if k["lane"] == 4 else 496) if layout.endswith("widest") else -1
    k["hs"] = STRIP_LAYOUTS[layout] if strips else (-1 if layout == "auto" else -2)
    say(f"one-pass {nx}x{ny} {layout}")
    got, tr, info = gpu(adw, k, True)
    if layout.endswith("widest"):
        assert info["fused_tile_cols"] == widest(nx, 240 if k["lane"] == 4 else 496)
    if k["lane"] > 0:
        assert info["fused_lane_nodes"] == k["lane"]
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    assert info["fused_segment_rows"] == (k["hs"] if strips else auto_plan(nx, ny, ncu)[2] if layout == "auto" else 0)
    if strips:
        assert info["fused_lane_nodes"] == 4 and info["fused_tile_cols"] == widest(nx, 240)
        assert info["fused_tiles"] == -(-nx // info["fused_tile_cols"]) * -(-ny // k["hs"])
    ref, rtr = oracle(oracle_lib, k)
    check(got, ref, what="level")
    check(tr, rtr, what="traces")


TOL64, TOL64_MAX = 1e-12, 1e-11
F64_STRIP_LAYOUTS = {"auto": -1, "strips_h8": 8, "strips_h30": 30, "strips_h1000": 1000}


@pytest.mark.parametrize("nx,ny", [(480, 64), (488, 65), (1000, 700), (960, 130), (64, 64), (2048, 300),
                                   (4, 200), (1504, 33), (64, 1), (40, 3), (194, 90)])
@pytest.mark.parametrize("layout", sorted(F64_STRIP_LAYOUTS))
def test_one_pass_f64_matches_oracle(adw, oracle_lib, nx, ny, layout):
    """The FP64 one-pass step (column strips of at most 64 columns, 16 halo columns and
    rows, truncation bound 4 qs^17 below 2^-53) against the FP64 oracle after 30 steps
    with two point sources and six receivers: relative L2 <= 1e-12 and max-norm
    <= 1e-11 (level and traces); the plan's automatic strips and 8-, 30- and 1000-row
    segments (bands cut anywhere, segments shorter than a band, longer than the grid)."""
    k = case(nx, ny, seed=nx + 7 * ny, f64=True)
    k["lane"], k["tile_cols"], k["hs"] = 0, -1, F64_STRIP_LAYOUTS[layout]
    say(f"one-pass f64 {nx}x{ny} {layout}")
    got, tr, info = gpu(adw, k, True)
    assert info["fused_step"] == 1 and info["fused_segment_rows"] > 0 and info["fused_tile_cols"] <= 64
    if layout != "auto":
        assert info["fused_segment_rows"] == k["hs"]
    ref, rtr = oracle(oracle_lib, k)
    check(got, ref, TOL64, TOL64_MAX, "level")
    check(tr, rtr, TOL64, TOL64_MAX, "traces")


def test_one_pass_f64_forced_widths_agree(adw, oracle_lib):
    """FP64 strips forced to 16, 40 and 64 columns (one width each) and the automatic
    mix reach the oracle's level to the FP64 bars on a 1000 x 700 grid."""
    k = case(1000, 700, seed=12, f64=True, nsteps=20)
    ref, _ = oracle(oracle_lib, k)
    for wt in (16, 40, 64, -1):
        k["lane"], k["tile_cols"], k["hs"] = 0, wt, -1 if wt == -1 else 200
        say(f"one-pass f64 width {wt}")
        got, _, info = gpu(adw, k, True)
        if wt > 0:
            assert info["fused_tile_cols"] == wt and info["fused_strips_wide"] == -(-1000 // wt)
        check(got, ref, TOL64, TOL64_MAX, f"width {wt}")


def test_one_pass_f64_short_segments(adw, oracle_lib):
    """FP64 strips of 64 columns forced to segments of 8, 17, 63 and 100 rows: 2, 3, 4
    and 6 bands a segment, so the pass count of the y-role split by stage (bands + 2)
    takes both parities and the first and last bands meet; each reaches the oracle's
    level to the FP64 bars on a 300 x 260 grid."""
    k = case(300, 260, seed=14, f64=True, nsteps=12)
    ref, _ = oracle(oracle_lib, k)
    for hs in (8, 17, 63, 100):
        k["lane"], k["tile_cols"], k["hs"] = 0, 64, hs
        say(f"one-pass f64 segments of {hs} rows")
        got, _, info = gpu(adw, k, True)
        assert info["fused_tile_cols"] == 64 and info["fused_segment_rows"] == hs
        check(got, ref, TOL64, TOL64_MAX, f"segments of {hs}")


def test_one_pass_mixed_strip_widths(adw, oracle_lib):
    """4096 x 3600: the automatic plan takes 18 column strips, 8 of 232 and 10 of 224
    columns, 14 segments of 258 rows; 3 steps against the oracle (relative L2 and
    max-norm), including the traces."""
    nx, ny = 4096, 3600
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    sp = strip_plan(nx, ny, ncu)
    if sp is None:
        pytest.skip(f"no column-strip plan for {ncu} compute units")
    k = case(nx, ny, seed=31, nsteps=3)
    k["lane"], k["tile_cols"], k["hs"] = -1, -1, -1
    say(f"one-pass mixed strip widths {nx}x{ny}")
    got, tr, info = gpu(adw, k, True)
    assert (info["fused_tile_cols"], info["fused_segment_rows"], info["fused_strips_wide"]) == (sp[0], sp[3], sp[2])
    assert info["fused_tiles"] == sp[1] * -(-ny // sp[3])
    ref, rtr = oracle(oracle_lib, k)
    check(got, ref, what="level")
    check(tr, rtr, what="traces")


def test_one_pass_equals_two_pass_on_gpu(adw):
    k = case(1024, 1024, cfl=0.5, seed=9, nsteps=60)
    say("one-pass vs two-pass 1024^2")
    a, ta, _ = gpu(adw, k, True)
    b, tb, _ = gpu(adw, k, False)
    check(a, b, 3e-6, 3e-6, "level")
    check(ta, tb, 3e-6, 3e-6, "traces")


@pytest.mark.parametrize("lane", [8, 4, "strips"])
def test_one_pass_near_the_bound(adw, oracle_lib, lane):
    """r_max = 0.17, just inside the bound (the truncation is then closest to 2^-24)."""
    nx = ny = 512
    h = 1.0 / 513
    dt = np.sqrt(2 * 0.17) * h / 3.0
    k = case(nx, ny, seed=5, nsteps=80)
    k["dt"] = dt
    k["lane"], k["hs"] = (0, 100) if lane == "strips" else (lane, -2)
    say(f"one-pass near bound {lane}")
    got, tr, info = gpu(adw, k, True)
    assert 0.165 < info["r_max"] < 0.175
    ref, rtr = oracle(oracle_lib, k)
    check(got, ref, what="level")
    check(tr, rtr, what="traces")


@pytest.mark.parametrize("lane", [8, 4, "strips"])
def test_one_pass_many_sources_in_a_tile(adw, oracle_lib, lane):
    """More point sources in one tile than it stages (read from memory instead),
    including repeated nodes."""
    k = case(480, 64, seed=11, nsteps=20, nsrc=40)
    k["lane"], k["hs"] = (0, 64) if lane == "strips" else (lane, -2)
    k["src_idx"][5] = k["src_idx"][3]
    say("one-pass 40 sources")
    got, tr, _ = gpu(adw, k, True)
    ref, rtr = oracle(oracle_lib, k)
    check(got, ref, what="level")
    check(tr, rtr, what="traces")


def test_tile_width_plan(adw):
    """The plan: column strips where each compute unit gets a segment of at least 256
    rows, else tiles balanced over the compute units; widths, lanes and segment rows
    can be forced and set back to automatic; bad values are rejected."""
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    for n in (8192, 6144, 4096, 2048, 1024):
        w = adw.Wave(n, n, 1.0 / (n + 1), 0.5 / (n + 1), c=1.0, dtype=torch.float32)
        i = w.info()
        lane, wt, hs = auto_plan(n, n, ncu)
        assert (i["fused_lane_nodes"], i["fused_tile_cols"], i["fused_segment_rows"]) == (lane, wt, hs), (n, i)
        sp = strip_plan(n, n, ncu)
        tx = sp[1] if sp else -(-n // wt)
        assert i["fused_tiles"] == tx * -(-n // (hs if hs else 64))
        if sp:
            assert i["fused_strips_wide"] == sp[2]
        w.set_tuning(fused_lane_nodes=8, fused_tile_cols=488)
        j = w.info()
        assert j["fused_tile_cols"] == 488 and j["fused_lane_nodes"] == 8 and j["fused_segment_rows"] == 0
        with pytest.raises(RuntimeError):
            w.set_tuning(fused_lane_nodes=4, fused_tile_cols=248)     # 4 nodes per lane: <= 240
        w.set_tuning(fused_lane_nodes=-1, fused_tile_cols=-1)
        j = w.info()
        assert (j["fused_lane_nodes"], j["fused_tile_cols"], j["fused_segment_rows"]) == (lane, wt, hs)
        for bad in (500, 100):
            with pytest.raises(RuntimeError):
                w.set_tuning(fused_tile_cols=bad)
        w.set_tuning(fused_segment_rows=100)
        j = w.info()
        assert (j["fused_lane_nodes"], j["fused_tile_cols"], j["fused_segment_rows"]) == (4, widest(n, 240), 100)
        assert j["fused_tiles"] == -(-n // widest(n, 240)) * -(-n // 100)
        w.set_tuning(fused_segment_rows=-2)
        assert w.info()["fused_segment_rows"] == 0
        w.set_tuning(fused_segment_rows=-1)
        j = w.info()
        assert (j["fused_lane_nodes"], j["fused_tile_cols"], j["fused_segment_rows"]) == (lane, wt, hs)
        for bad in ({"fused_segment_rows": 5}, {"fused_segment_rows": -3},
                    {"fused_segment_rows": 100, "fused_lane_nodes": 8},
                    {"fused_segment_rows": 100, "fused_tile_cols": 248}):
            with pytest.raises(RuntimeError):
                w.set_tuning(**bad)
        w.close()


def test_forced_widths_agree(adw):
    """Different tile and strip layouts truncate at different places: each stays
    within the bound of the exact step."""
    k = case(1000, 700, cfl=0.5, seed=4, nsteps=40)
    ref, rtr, _ = gpu(adw, k, False)
    for wt, lane, hs in ((64, 8, -2), (136, 8, -2), (256, 8, -2), (496, 8, -2), (64, 4, -2), (120, 4, -2),
                         (240, 4, -2), (64, 0, 40), (120, 0, 333), (240, 0, 8), (200, 0, 701)):
        k["tile_cols"] = wt
        k["lane"] = lane
        k["hs"] = hs
        say(f"one-pass 1000x700 width {wt}, {lane} nodes per lane, segment rows {hs}")
        got, tr, info = gpu(adw, k, True)
        assert info["fused_tile_cols"] == wt and info["fused_lane_nodes"] == (lane or 4)
        assert info["fused_segment_rows"] == max(hs, 0)
        check(got, ref, 3e-6, 3e-6, "level")
        check(tr, rtr, 3e-6, 3e-6, "traces")


@pytest.mark.parametrize("layout", ["lane8", "lane4", "strips"])
def test_one_step_truncation_bound(adw, oracle_lib, layout):
    """One step at r_max ~ 0.17 against the oracle's exact step, node by node.

    The one-pass step truncates each line solve where the decay factor qs of the
    line recurrences has fallen below 4 qs^9 <= 2^-24, so per step
      max |u_fused - u_exact| <= 4 qs^9 max|w| + (FP32 rounding of the step).
    u^{n-1} = 2 u^n makes u^{n+1} the increment d itself (2u^n - u^{n-1} = 0 exactly
    in FP32), so the comparison sees the line solves and not the rounding of a large
    level.  The FP32 allowance is the same step by the GPU's exact two-pass kernels,
    node by node against the oracle, plus one unit of rounding of max|d| (the two
    paths associate their sums differently)."""
    nx, ny = 720, 600
    h = 1.0 / 721
    rmax = 0.17
    dt = np.sqrt(2 * rmax) * h / 3.0
    rng = np.random.default_rng(17)
    c = wl.smooth_field(nx, ny, 1.0, 3.0, seed=17).astype(np.float32)
    uc = (wl.gaussian_pulse(nx, ny, sigma=0.05) + 0.1 * rng.standard_normal((ny, nx))).astype(np.float32)
    up = 2 * uc
    parts = oracle_lib.step_parts(c.astype(np.float64) ** 2, up, uc, h, dt)
    ref = parts["u_next"]
    lane, hs = {"lane8": (8, -2), "lane4": (4, -2), "strips": (0, 100)}[layout]

    def one(one_pass):
        wave = adw.Wave(nx, ny, h, dt, c=dev(c), dtype=torch.float32)
        wave.set_tuning(fused_step=one_pass, **(dict(fused_lane_nodes=lane, fused_segment_rows=hs)
                                                if one_pass else {}))
        info = wave.info()
        a, b = wave.step(dev(up), dev(uc), 1)
        torch.cuda.synchronize()
        out = b.cpu().numpy().astype(np.float64)
        wave.close()
        return out, info

    fused, info = one(True)
    exact, _ = one(False)
    assert info["fused_step"] == 1 and 0.165 < info["r_max"] < 0.175
    rm = float(info["r_max"])
    qs = (1 + 2 * rm - np.sqrt(1 + 4 * rm)) / (2 * rm)
    trunc = 4 * qs ** 9 * np.abs(parts["w"]).max()
    allowance = np.abs(exact - ref).max() + 2.0 ** -24 * np.abs(ref).max()
    err = np.abs(fused - ref).max()
    say(f"  one step {layout}: max|fused - exact oracle| {err:.3e}, bound {trunc:.3e} + FP32 {allowance:.3e}")
    assert err <= trunc + allowance


@pytest.mark.parametrize("hs", [100, -1])
def test_one_step_truncation_bound_f64(adw, oracle_lib, hs):
    """The FP64 one-pass step, one step at r_max ~ 0.13 (near the largest r its bound
    admits) against the oracle's exact step, node by node:
      max |u_fused - u_exact| <= 4 qs^17 max|w| + (FP64 rounding of the step),
    with u^{n-1} = 2 u^n as in the FP32 test (u^{n+1} is then the increment d).  At this
    precision the truncation (below half an ulp) is smaller than the roundings of the
    two paths, which associate the step's sums differently (the one-pass step runs
    the x-lines as scans of affine maps over 2-node lanes, the exact step over 8-node
    segments): the FP64 allowance is the GPU's exact two-pass step against the oracle
    plus four units of rounding of max|d| (measured: the exact step 1.5, the one-pass
    step 2.9).  Strips of 100 rows and the automatic plan."""
    nx, ny = 720, 600
    h = 1.0 / 721
    rmax = 0.13
    dt = np.sqrt(2 * rmax) * h / 3.0
    rng = np.random.default_rng(19)
    c = wl.smooth_field(nx, ny, 1.0, 3.0, seed=19)
    uc = wl.gaussian_pulse(nx, ny, sigma=0.05) + 0.1 * rng.standard_normal((ny, nx))
    up = 2 * uc
    parts = oracle_lib.step_parts(c ** 2, up, uc, h, dt)
    ref = parts["u_next"]

    def one(one_pass):
        wave = adw.Wave(nx, ny, h, dt, c=dev(c), dtype=torch.float64)
        wave.set_tuning(fused_step=one_pass, **(dict(fused_segment_rows=hs) if one_pass else {}))
        info = wave.info()
        a, b = wave.step(dev(up), dev(uc), 1)
        torch.cuda.synchronize()
        out = b.cpu().numpy()
        wave.close()
        return out, info

    fused, info = one(True)
    exact, _ = one(False)
    assert info["fused_step"] == 1 and 0.125 < info["r_max"] < 0.1331
    rm = float(info["r_max"])
    qs = (1 + 2 * rm - np.sqrt(1 + 4 * rm)) / (2 * rm)
    trunc = 4 * qs ** 17 * np.abs(parts["w"]).max()
    allowance = np.abs(exact - ref).max() + 4 * 2.0 ** -53 * np.abs(ref).max()
    err = np.abs(fused - ref).max()
    say(f"  one step f64 hs={hs}: max|fused - exact oracle| {err:.3e}, bound {trunc:.3e} + FP64 {allowance:.3e}")
    assert err <= trunc + allowance
