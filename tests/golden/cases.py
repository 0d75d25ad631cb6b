"""Inputs of the stored reference values in this folder (no arithmetic of the
method here: the problems come from the seeded generators in workloads.py).

Each case names the problem, the nodes whose final values are stored and, where
the run has receivers, their nodes; make_golden.py runs the oracle on them and
writes one text file per case."""
import numpy as np

from paper_2006_10142_amd import workloads as wl


def sample_nodes(nx: int, ny: int, count: int = 40) -> np.ndarray:
    """Evenly spread flat node offsets, plus the centre node and the four corners."""
    spread = np.linspace(0, nx * ny - 1, count).round().astype(np.int64)
    extra = np.array([(ny // 2) * nx + nx // 2, 0, nx - 1, (ny - 1) * nx, nx * ny - 1])
    return np.unique(np.concatenate([spread, extra])).astype(np.int32)


def c1_standing_wave():
    """C1 in full: 128^2 interior nodes, h = 1/129, dt = h/2, kappa = 1,
    u0 = sin(pi x) sin(pi y), psi = 0, f = 0, ghost start, 200 steps, FP64."""
    p = wl.config_c1()
    return p, sample_nodes(p.nx, p.ny)


def c3_small(dtype: str):
    """The C3 recipe on a 96^2 grid: per-node speed in [1, 3] (seed 3), dt = 0.4 h /
    max c, zero initial levels, Ricker (f0 = 10) at the centre node, 120 steps (past
    the wavelet's peak at t = 0.1), with 8 receivers on a ring around the source.
    dtype "f32" rounds the inputs to FP32 once (the oracle then runs in FP64 on
    those values)."""
    p = wl.config_c3(dtype=dtype, nsteps=120, n=96)
    n = p.nx
    ci = n // 2 - 1
    ring = [(ci + dy, ci + dx) for dy, dx in
            ((-12, 0), (12, 0), (0, -12), (0, 12), (-9, -9), (9, 9), (-9, 9), (20, -3))]
    p.rec_idx = np.array([j * n + i for j, i in ring], np.int32)
    near = np.array([(ci + dy) * n + ci + dx for dy in range(-15, 16, 5) for dx in range(-15, 16, 5)])
    return p, np.unique(np.concatenate([sample_nodes(p.nx, p.ny), near])).astype(np.int32)


def tridiag_systems():
    """Strictly diagonally dominant systems of sizes 1, 2, 7 and 33 (seeded), with
    a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k]."""
    out = []
    for n, seed in ((1, 1), (2, 2), (7, 3), (33, 4)):
        rng = np.random.default_rng(seed)
        a = rng.uniform(-1, 1, n)
        c = rng.uniform(-1, 1, n)
        b = (np.abs(a) + np.abs(c) + rng.uniform(0.1, 1.0, n)) * rng.choice([-1.0, 1.0], n)
        d = rng.standard_normal(n)
        out.append((n, a, b, c, d))
    return out


def _lines_in_window(n, rows, cols, lo, hi, every):
    """Flat offsets of the given full rows and columns, restricted to [lo, hi) along
    the line and taken every `every` nodes."""
    along = np.arange(lo, hi, every)
    out = [r * n + along for r in rows] + [along * n + c for c in cols]
    return np.concatenate(out)


def c3p_full():
    """C3p at its full size: the C3 speed field on 8192^2 (FP32 inputs), Gaussian u0
    (sigma 0.02) with the ghost start, 500 steps.  After 500 steps the wave has moved
    about 0.02 from the pulse, so the stored nodes sit in the window of +-1024 nodes
    around the centre: whole rows and columns (every other node) where the line
    partitions of the solver meet -- rows at multiples of 1171 (3512|3513, 4683|4684)
    and 32 (3583|3584), columns at multiples of 240 (3839|3840, 4079|4080, 4319|4320)
    -- plus the centre row, 2048 seeded random nodes of the window and the evenly
    spread far-field sample."""
    p = wl.config_c3p(dtype="f32", nsteps=500)
    n = p.nx
    lines = _lines_in_window(n, rows=(3512, 3513, 3583, 3584, 4095, 4683, 4684),
                             cols=(3839, 3840, 4079, 4080, 4319, 4320), lo=3072, hi=5120, every=2)
    rng = np.random.default_rng(81)
    rnd = rng.integers(3072, 5120, size=(2048, 2))
    rnd = rnd[:, 0] * n + rnd[:, 1]
    return p, np.unique(np.concatenate([lines, rnd, sample_nodes(n, n)])).astype(np.int32)


def c3_full():
    """C3 at its full size (the benchmark's workload): 8192^2 speed field in [1, 3]
    (FP32 inputs), zero initial levels, Ricker (f0 = 10) at the centre node, 500 steps.
    The wavelet has only begun after 500 steps (t = 8.1e-3 against its peak at 0.1) and
    the wave has moved at most about 200 nodes, so the stored nodes are the source row
    and column over +-400 nodes, 1024 seeded random nodes within +-300 of the source,
    and the evenly spread far-field sample."""
    p = wl.config_c3(dtype="f32", nsteps=500)
    n = p.nx
    ci = n // 2 - 1
    lines = _lines_in_window(n, rows=(ci,), cols=(ci, 4080), lo=ci - 400, hi=ci + 401, every=1)
    rng = np.random.default_rng(82)
    rnd = rng.integers(ci - 300, ci + 301, size=(1024, 2))
    rnd = rnd[:, 0] * n + rnd[:, 1]
    return p, np.unique(np.concatenate([lines, rnd, sample_nodes(n, n)])).astype(np.int32)


CASES = {
    "c1_standing_wave_128_f64": lambda: c1_standing_wave(),
    "c3_recipe_96_f64": lambda: c3_small("f64"),
    "c3_recipe_96_f32_inputs": lambda: c3_small("f32"),
}

# full-size runs (minutes of oracle time each; written once, compared on the GPU only)
FULL = {
    "c3p_pulse_8192_500_f32_inputs": lambda: c3p_full(),
    "c3_ricker_8192_500_f32_inputs": lambda: c3_full(),
}
