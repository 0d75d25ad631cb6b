"""Readers of the stored reference values in this folder (plain text; no oracle)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name: str):
    """(level offsets, level values, receiver offsets or None, traces (nsteps, nrec) or None)"""
    offs, vals, recs, tr = [], [], None, {}
    with open(os.path.join(HERE, name + ".txt")) as fh:
        for line in fh:
            if line.startswith("# receiver-nodes "):
                recs = np.array([int(v) for v in line.split()[2:]], np.int32)
            elif line.startswith("level "):
                _, k, v = line.split()
                offs.append(int(k))
                vals.append(float(v))
            elif line.startswith("trace "):
                _, k, r, v = line.split()
                tr[(int(k), int(r))] = float(v)
    traces = None
    if tr:
        nk = 1 + max(k for k, _ in tr)
        nr = 1 + max(r for _, r in tr)
        traces = np.array([[tr[(k, r)] for r in range(nr)] for k in range(nk)])
    return np.array(offs, np.int64), np.array(vals), recs, traces


def load_tridiag():
    systems, cur = [], None
    with open(os.path.join(HERE, "tridiag_small_f64.txt")) as fh:
        for line in fh:
            if line.startswith("system "):
                cur = []
                systems.append(cur)
            elif line.startswith("row "):
                cur.append([float(v) for v in line.split()[2:]])
    return [np.array(s) for s in systems]
