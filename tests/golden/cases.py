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


CASES = {
    "c1_standing_wave_128_f64": lambda: c1_standing_wave(),
    "c3_recipe_96_f64": lambda: c3_small("f64"),
    "c3_recipe_96_f32_inputs": lambda: c3_small("f32"),
}
