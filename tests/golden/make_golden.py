"""Writes the stored reference values of this folder from the oracle (and only
the oracle): python -m tests.golden.make_golden (from the repository root).

Every file states what it follows; the scheme is eq. (CN1) of the paper in the
factored delta form (x-lines, then y-lines, then the update), with the ghost
start level and point sources f^n at node offsets, receivers sampling each new
level."""
import os

import numpy as np

import oracle
from tests.golden import cases
from tests.golden.store import HERE

HEAD = {
    "c1_standing_wave_128_f64":
        "C1: the standing wave sin(pi x) sin(pi y) on 128^2 interior nodes, 200 steps.\n"
        "Follows eq. (CN1) as the factored delta form (x-lines, y-lines, update), the\n"
        "ghost start level and the zero Dirichlet walls.  The discrete closed form\n"
        "cos((n+1) theta) sin(pi x) sin(pi y) also gives these values (checked on load).",
    "c3_recipe_96_f64":
        "The C3 recipe at 96^2: per-node speed, Ricker point source at the centre, 120\n"
        "steps, 8 receivers.  Follows eq. (CN1) as the factored delta form with a\n"
        "per-node coefficient kappa = c^2 in each line equation, point sources f^n and\n"
        "receivers sampling each new level.",
    "c3_recipe_96_f32_inputs":
        "As c3_recipe_96_f64, with the speed field and source values rounded to FP32\n"
        "once; the oracle runs in FP64 on those values (the FP32 parity inputs).",
    "c3p_pulse_8192_500_f32_inputs":
        "C3p in full: the C3 speed field on 8192^2 nodes, Gaussian u0 (sigma 0.02), ghost\n"
        "start, 500 steps, inputs rounded to FP32 once and run in FP64.  Follows eq. (CN1)\n"
        "as the factored delta form with a per-node coefficient kappa = c^2.  Nodes: rows\n"
        "and columns where the solver's line partitions meet, the centre row, random nodes\n"
        "near the pulse and a far-field sample.",
    "c3_ricker_8192_500_f32_inputs":
        "C3 in full: 8192^2 speed field in [1, 3], zero initial levels, Ricker point\n"
        "source (f0 = 10) at the centre node, 500 steps, inputs rounded to FP32 once and\n"
        "run in FP64.  Follows eq. (CN1) as the factored delta form with point sources f^n.\n"
        "Nodes: the source row and columns, random nodes near the source, a far-field sample.",
}


def write_run(name: str):
    p, nodes = {**cases.CASES, **cases.FULL}[name]()
    _, uc, tr = oracle.run_problem(p)
    lines = [f"# {l}" for l in HEAD[name].splitlines()]
    lines += ["# Written by tests/golden/make_golden.py from the oracle; do not edit by hand.",
              f"# problem {p.name}: nx={p.nx} ny={p.ny} h={p.h!r} dt={p.dt!r} nsteps={p.nsteps} dtype={p.dtype}",
              f"# section level: final level u^(n+nsteps) at {nodes.size} flat node offsets (j*nx+i)",
              "# level <offset> <value>"]
    flat = uc.ravel()
    lines += [f"level {int(k)} {float(flat[k])!r}" for k in nodes]
    if tr is not None and p.rec_idx.size:
        lines.append("# section trace: receiver values, step k (0-based) of the run, receiver r")
        lines.append("# receiver-nodes " + " ".join(str(int(r)) for r in p.rec_idx))
        lines.append("# trace <k> <r> <value>")
        for k in range(tr.shape[0]):
            lines += [f"trace {k} {r} {float(tr[k, r])!r}" for r in range(tr.shape[1])]
    with open(os.path.join(HERE, name + ".txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def write_tridiag():
    lines = ["# Batched tridiagonal solves (the line systems' solver): strictly diagonally",
             "# dominant systems a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k], solved by the",
             "# Thomas elimination (no pivoting), one system per 'system' line.",
             "# Written by tests/golden/make_golden.py from the oracle; do not edit by hand.",
             "# system <n>, then for k = 0..n-1: row <k> <a> <b> <c> <d> <x>"]
    for n, a, b, c, d in cases.tridiag_systems():
        x = oracle.thomas(a, b, c, d)
        lines.append(f"system {n}")
        lines += ["row %d %r %r %r %r %r" % (k, float(a[k]), float(b[k]), float(c[k]), float(d[k]), float(x[k]))
                  for k in range(n)]
    with open(os.path.join(HERE, "tridiag_small_f64.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    import sys
    oracle.build()
    # optional names select cases (the full-size ones take minutes each)
    names = sys.argv[1:] or list(cases.CASES) + list(cases.FULL)
    for name in names:
        if name == "tridiag":
            write_tridiag()
        else:
            print("writing", name, flush=True)
            write_run(name)
    if not sys.argv[1:]:
        write_tridiag()
    print("written:", sorted(f for f in os.listdir(HERE) if f.endswith(".txt")))
