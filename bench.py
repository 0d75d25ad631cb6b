"""Benchmark of the ADI wave step on one MI355X.

Workload (default): the 8192^2 FP32 heterogeneous case -- per-node wave speed
in [1, 3] (16 seeded Gaussian bumps), dt = 0.4 h / max c, Ricker point source
(f0 = 10) at the centre node, zero initial levels.  A "step" is one full ADI
time step: right-hand side + x-line solves + y-line solves + update.

Prints ONE JSON line:
  value       Mpts/s = nx*ny*steps / t_timed / 1e6 (inputs resident in HBM)
  roofline    dominant kernel: algorithmic bytes per launch / its mean duration
              (HIP events around every launch on the solver's stream)
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpts/s per ADI step + HBM GB/s (% peak); batched & adjoint vs plain, same GPU"
HBM_PEAK_GBPS = 8000.0
# The paper's own timings (Table 1: total seconds for 50 FP64 time steps of its
# cyclic-reduction ADI solver on an RTX 2080 Ti with an i7-9800X host), converted
# to Mpts/s per step.  Context only: other hardware, precision and solver design.
PAPER_TABLE1 = {
    "source": "Table 1, 50 FP64 steps, c = 1; RTX 2080 Ti + i7-9800X (3.8 GHz)",
    "unit": "Mpts/s per step",
    "8192x8192": {"cpu": 1.03, "gpu": 7.70, "gpu_openmp": 14.01, "gpu_openmp_mpi_8_cores": 21.04},
    "2048x2048": {"cpu": 1.11, "gpu": 4.66, "gpu_openmp": 4.66, "gpu_openmp_mpi_8_cores": 6.93},
}

# Algorithmic bytes per grid node per launch (element size E, per-node coefficient):
#   x_sweep_rhs     reads u^n and r, writes w                      3E
#   y_solve_update  reads w, r, u^n, u^{n-1}, writes u^{n+1}       5E
#   y_reduce        reads w and r                                  2E
#   x_sweep_rhs_y_reduce  the x-sweep with the y-chunk elimination fused: 3E
# The whole step's two-pass minimum is 8E (32 B/node in FP32).
#   fused_step      the one-pass step: reads u^n, r, u^{n-1}, writes u^{n+1}  4E
ALG_BYTES_PER_NODE = {"x_sweep_rhs": 3, "x_sweep_rhs_y_reduce": 3, "y_solve_update": 5,
                      "y_reduce": 2, "fused_step": 4}
STEP_BYTES_PER_NODE = 8          # two-pass step
FUSED_STEP_BYTES_PER_NODE = 4    # one-pass step

WORKLOADS = {
    "c3": ("c3_heterogeneous_ricker_8192x8192_f32", "f32", 8192),
    "c2f32": ("c2_gaussian_pulse_2048x2048_f32", "f32", 2048),
    "c2f64": ("c2_gaussian_pulse_2048x2048_f64", "f64", 2048),
}


def kernel_source_hash() -> str:
    """Hash of the sources that define the plain step's kernels and their launches
    (the batched and adjoint forms live in their own headers)."""
    h = hashlib.sha256()
    for f in ("adiwave.hip", "kernels.hpp", "line_solver.hpp", "xsweep.hpp", "fused.hpp", "fused4.hpp", "fusedr.hpp"):
        with open(os.path.join(ROOT, "paper_2006_10142_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str, launches_bytes: float):
    """HBM traffic from the committed counter summary, if it matches the current source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        ent = data.get(workload, {}).get(kernel)
        if not ent or ent.get("source_hash") != kernel_source_hash():
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def make_problem(key: str, nsteps: int):
    from paper_2006_10142_amd import workloads as wl
    if key == "c3":
        return wl.config_c3(dtype="f32", nsteps=nsteps)
    if key == "c2f32":
        return wl.config_c2(dtype="f32", nsteps=nsteps)
    return wl.config_c2(dtype="f64", nsteps=nsteps)


def cpu_baseline(prob, steps: int):
    """FP64 oracle on a bounded sample: `steps` ADI steps of the same workload."""
    import numpy as np
    import oracle
    oracle.build()
    kappa = prob.kappa_field()
    if prob.u_curr is not None:
        up = np.asarray(prob.u_prev, np.float64)
        uc = np.asarray(prob.u_curr, np.float64)
    else:
        up = np.asarray(prob.u0, np.float64)
        uc = up.copy()
    amp = None if prob.src_amp is None else np.asarray(prob.src_amp)[:steps]
    si = prob.src_idx if prob.src_idx.size else None
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.run(kappa, up, uc, prob.h, prob.dt, steps, src_idx=si, src_amp=amp, threads=cores)
    t = time.perf_counter() - t0
    # one host thread, on a 2048 x 2048 corner of the same fields (one step)
    n1 = min(2048, prob.nx, prob.ny)
    k1 = np.ascontiguousarray(np.broadcast_to(kappa, (prob.ny, prob.nx))[:n1, :n1]) \
        if np.ndim(kappa) else kappa
    t1 = time.perf_counter()
    oracle.run(k1, np.ascontiguousarray(up[:n1, :n1]), np.ascontiguousarray(uc[:n1, :n1]), prob.h, prob.dt, 1,
               threads=1)
    t1 = time.perf_counter() - t1
    return {"value": round(prob.nx * prob.ny * steps / t / 1e6, 2), "unit": "Mpts/s",
            "cores": cores, "kind": "oracle",
            "build": "gcc -O2 -fopenmp -ffp-contract=off, no -march; OpenMP over lines; x-lines "
                     "row by row, y-lines one column at a time (stride nx); untuned",
            "sample": f"{steps} ADI steps of the same {prob.nx}x{prob.ny} workload, FP64, "
                      f"{t:.1f} s wall",
            "one_thread": {"value": round(n1 * n1 / t1 / 1e6, 2), "unit": "Mpts/s",
                           "sample": f"1 step of a {n1}x{n1} corner of the same fields, FP64, {t1:.1f} s"},
            "cpu_model": cpu_model()}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_batched(adw, torch, steps: int, warmup: int, plain_value: float):
    """C4: 256 independent FP32 simulations (N in 256..1024), one launch per kernel per
    step for the whole batch, autotuned plan, replayed hipGraph."""
    import numpy as np
    from paper_2006_10142_amd import workloads as wl
    probs = wl.config_c4(dtype="f32", nsteps=steps)
    dev = torch.device("cuda:0")
    b = adw.Batch([(p.nx, p.ny) for p in probs], [p.h for p in probs], [p.dt for p in probs],
                  [torch.from_numpy(p.c).to(dev) for p in probs], dtype=torch.float32)
    u0 = [torch.from_numpy(np.ascontiguousarray(p.u0)).to(dev) for p in probs]
    u1 = [torch.zeros_like(x) for x in u0]
    tuned_ms = b.autotune(trial_steps=5)
    b.bind(u0, u1)
    b.start("ghost")
    b.graph(True)
    b.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, curr = b.levels()
    finite = all(bool(torch.isfinite(x).all()) for x in curr)
    plan = b.plan()
    nodes = plan["nodes"]
    value = nodes * steps / (ms / 1e3) / 1e6
    b.close()
    return {"workload": "c4_batch_256_sims_256_to_1024_f32", "value": round(value, 1),
            "unit": "Mpts/s", "ms_per_step": round(ms / steps, 5), "sims": len(probs),
            "nodes_per_step": nodes, "steps": steps, "graph": True,
            "plan": {k: plan[k] for k in ("x_threads_per_line", "x_grid", "yscan_grid",
                                          "ysolve_grid", "fused_lane_nodes", "fused_strips")},
            "autotune_ms_per_step": round(tuned_ms, 5),
            "step": "one-pass" if plan["fused_step"] else "two-pass",
            "step_algorithmic_bytes_per_node": 4 * (FUSED_STEP_BYTES_PER_NODE if plan["fused_step"]
                                                    else STEP_BYTES_PER_NODE),
            "step_algorithmic_GBps": round((FUSED_STEP_BYTES_PER_NODE if plan["fused_step"] else STEP_BYTES_PER_NODE)
                                           * 4 * nodes * steps / (ms / 1e3) / 1e9, 1),
            "vs_plain": round(value / plain_value, 4), "finite": finite}


def bench_tridiag(adw, torch, n: int = 8192, batch: int = 8192, reps: int = 5):
    """The ABI's batched general line solve on random strictly diagonally dominant FP32
    systems: n unknowns, batch systems, contiguous (system after system) and interleaved
    (unknown k of every system side by side).  Algorithmic bytes per unknown: a, b, c, d
    read and d written (20 B)."""
    out = {}
    g = torch.Generator(device="cuda").manual_seed(7)
    total = n * batch
    a = torch.rand(total, device="cuda", generator=g) - 0.5
    c = torch.rand(total, device="cuda", generator=g) - 0.5
    b = a.abs() + c.abs() + 0.5
    d0 = torch.rand(total, device="cuda", generator=g)
    for layout, ss, es in (("contiguous", n, 1), ("interleaved", 1, batch)):
        d = d0.clone()
        adw.tridiag_solve_batched(a, b, c, d, n, batch, ss, es)      # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            adw.tridiag_solve_batched(a, b, c, d, n, batch, ss, es)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbps = 20 * total / (ms / 1e3) / 1e9
        out[layout] = {"n": n, "batch": batch, "ms": round(ms, 4), "algorithmic_GBps": round(gbps, 1),
                       "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4),
                       "finite": bool(torch.isfinite(d).all().item())}
    del a, b, c, d0
    torch.cuda.empty_cache()
    return out


def bench_cr(adw, torch, prob, steps: int, plain_value: float):
    """The paper's line solver (cyclic reduction, one launch per level for all lines of
    a sweep) on the same workload, same GPU: a short timed run."""
    import numpy as np
    dev = torch.device("cuda:0")
    wave = adw.Wave(prob.nx, prob.ny, prob.h, prob.dt, dtype=torch.float32,
                    c=torch.from_numpy(prob.c).to(dev) if prob.c is not None else prob.c_scalar)
    if prob.u_curr is not None:
        a = torch.from_numpy(np.ascontiguousarray(prob.u_prev)).to(dev)
        b = torch.from_numpy(np.ascontiguousarray(prob.u_curr)).to(dev)
    else:
        a = torch.from_numpy(np.ascontiguousarray(prob.u0)).to(dev)
        b = wave.start(a)
    wave.set_tuning(cyclic_reduction=True)
    warm, kw = {}, {}
    if prob.src_amp is not None:
        si = torch.from_numpy(prob.src_idx).to(dev)
        amp = torch.from_numpy(np.ascontiguousarray(prob.src_amp[:steps + 2])).to(dev)
        warm, kw = dict(src_idx=si, src_amp=amp[:2]), dict(src_idx=si, src_amp=amp[2:])
    a, b = wave.step(a, b, 2, **warm)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    a, b = wave.step(a, b, steps, **kw)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    info = wave.info()
    wave.close()
    value = prob.nx * prob.ny * steps / (ms / 1e3) / 1e6
    return {"solver": "cyclic reduction, one launch per level, all lines of a sweep per launch",
            "value": round(value, 1), "unit": "Mpts/s", "ms_per_step": round(ms / steps, 4),
            "steps": steps, "launches_per_step": info["kernels_per_step"],
            "default_over_cr": round(plain_value / value, 2),
            "finite": bool(torch.isfinite(b).all())}


def bench_adjoint(adw, torch):
    """C5: dJ/dkappa of a receiver misfit on 1024^2 FP32, 2000 steps, checkpoints every 100
    steps, 64 receivers; target traces from the run on the second kappa field.

    Algorithmic bytes per node (E = 4 B), each launch's own inputs and outputs once:
      forward step   4E   the handle's step, the one-pass step here (8E where it takes the
                          exact two-pass step), plus 4E / K for the checkpoint copy every K
                          steps;
      backward step 21E   the recomputed step (the exact two-pass step, 8E), the transposed
                          y-lines (reads lambda, r, writes z: 3E) and the transposed x-lines
                          with the update folded in (reads z, r, two lambda levels, three u
                          levels, dJ/dkappa; writes dJ/dkappa and lambda: 10E; t stays on
                          chip, and w^k = A_y d^k is formed from the u levels).
    vs_plain divides by the plain solver's rate on the same 1024^2 grid (same kappa,
    source and step count; the handle's default step)."""
    import numpy as np
    from paper_2006_10142_amd import workloads as wl
    p, kt = wl.config_c5(dtype="f32")
    dev = torch.device("cuda:0")
    K = 100
    wave = adw.Wave(p.nx, p.ny, p.h, p.dt, dtype=torch.float32, kappa=torch.from_numpy(kt).to(dev))
    si = torch.from_numpy(p.src_idx).to(dev)
    ri = torch.from_numpy(p.rec_idx).to(dev)
    amp = torch.from_numpy(p.src_amp).to(dev)
    zero = torch.zeros((p.ny, p.nx), dtype=torch.float32, device=dev)
    target = wave.adjoint_forward(zero, zero, p.nsteps, src_idx=si, src_amp=amp, rec_idx=ri,
                                  checkpoint_every=K)
    wave.set_kappa(torch.from_numpy(p.kappa).to(dev))
    # warm-up pass (allocates the checkpoint and segment storage)
    tr = wave.adjoint_forward(zero, zero, p.nsteps, src_idx=si, src_amp=amp, rec_idx=ri,
                              checkpoint_every=K)
    wave.adjoint_backward(2.0 * (tr - target), src_idx=si, src_amp=amp, rec_idx=ri)
    torch.cuda.synchronize()
    fw, bw = [], []
    for _ in range(3):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        tr = wave.adjoint_forward(zero, zero, p.nsteps, src_idx=si, src_amp=amp, rec_idx=ri,
                                  checkpoint_every=K)
        e[1].record()
        gk, _ = wave.adjoint_backward(2.0 * (tr - target), src_idx=si, src_amp=amp, rec_idx=ri)
        e[2].record()
        torch.cuda.synchronize()
        fw.append(e[0].elapsed_time(e[1]))
        bw.append(e[1].elapsed_time(e[2]))
    fwd, bwd = float(np.median(fw)), float(np.median(bw))
    loss = float(((tr - target) ** 2).sum())
    finite = bool(torch.isfinite(gk).all())
    # the plain solver on the same grid, coefficient, source and step count
    a, b = zero.clone(), zero.clone()
    a, b = wave.step(a, b, 20, src_idx=si, src_amp=amp[:20])
    pl = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.zero_(); b.zero_()
        torch.cuda.synchronize()
        e0.record()
        a, b = wave.step(a, b, p.nsteps, src_idx=si, src_amp=amp)
        e1.record()
        torch.cuda.synchronize()
        pl.append(e0.elapsed_time(e1))
    plain_ms = float(np.median(pl))
    plain_step = "one-pass" if wave.info()["fused_step"] else "two-pass"
    nodes = p.nx * p.ny
    value = nodes * p.nsteps / ((fwd + bwd) / 1e3) / 1e6
    plain_value = nodes * p.nsteps / (plain_ms / 1e3) / 1e6
    E = 4
    fwd_e = 4 if wave.info()["fused_step"] else 8
    fb = (fwd_e + 4.0 / K) * E * nodes
    bb = 21 * E * nodes
    f_gbps = fb * p.nsteps / (fwd / 1e3) / 1e9
    b_gbps = bb * p.nsteps / (bwd / 1e3) / 1e9
    wave.close()
    return {"workload": "c5_adjoint_1024x1024_f32_2000_steps_64_receivers", "value": round(value, 1),
            "unit": "Mpts/s (gradient evaluation: forward with checkpoints + reverse pass)",
            "forward_ms": round(fwd, 3), "backward_ms": round(bwd, 3),
            "ms_per_step_forward": round(fwd / p.nsteps, 5),
            "ms_per_step_backward": round(bwd / p.nsteps, 5), "checkpoint_every": K,
            "forward_step": "one-pass" if fwd_e == 4 else "two-pass", "recompute_step": "two-pass",
            "algorithmic_bytes_per_node": {"forward_step": round((fwd_e + 4.0 / K) * E, 2), "backward_step": 21 * E},
            "roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBPS,
                         "forward": {"achieved": round(f_gbps, 1), "frac": round(f_gbps / HBM_PEAK_GBPS, 4)},
                         "backward": {"achieved": round(b_gbps, 1), "frac": round(b_gbps / HBM_PEAK_GBPS, 4)}},
            "loss": loss, "finite": finite,
            "plain_same_grid": {"value": round(plain_value, 1), "unit": "Mpts/s", "ms": round(plain_ms, 3),
                                "step": plain_step},
            "vs_plain": round(value / plain_value, 4)}


def plain_leg(adw, torch, prob, name: str, dtype: str, steps: int, warmup: int, reps: int,
              profile_steps: int, both: bool = True):
    """One plain-solver workload: create, initial levels, then the measured step (the
    handle's default: the one-pass step where allowed) and, with both=True and the
    one-pass step on, the exact two-pass step too.  Returns (main, two_pass or None,
    create_ms).  Each measurement: `warmup` untimed steps, then `reps` repetitions of
    exactly `steps` steps bracketed by synchronisation (the median is the figure), then
    per-kernel durations from events around every launch on the solver's stream."""
    import numpy as np
    tdt = torch.float32 if dtype == "f32" else torch.float64
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    wave = adw.Wave(prob.nx, prob.ny, prob.h, prob.dt, dtype=tdt,
                    c=torch.from_numpy(prob.c).to(dev) if prob.c is not None else prob.c_scalar)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    if prob.u_curr is not None:
        a = torch.from_numpy(np.ascontiguousarray(prob.u_prev)).to(dev)
        b = torch.from_numpy(np.ascontiguousarray(prob.u_curr)).to(dev)
    else:
        a = torch.from_numpy(np.ascontiguousarray(prob.u0)).to(dev)
        b = wave.start(a)
    src = {}
    if prob.src_amp is not None:
        amp = torch.from_numpy(np.ascontiguousarray(prob.src_amp)).to(dev)
        src = dict(src_idx=torch.from_numpy(prob.src_idx).to(dev))
    torch.cuda.synchronize()

    def srcs(first, count):
        if not src:
            return {}
        return dict(src, src_amp=amp[first:first + count])

    esz = 4 if dtype == "f32" else 8
    npts = prob.nx * prob.ny

    def measure(a, b):
        if warmup:
            a, b = wave.step(a, b, warmup, **srcs(0, warmup))
        torch.cuda.synchronize()
        reps_ms, walls = [], []
        for r in range(reps):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            ev0.record()
            a, b = wave.step(a, b, steps, **srcs(warmup + r * steps, steps))
            ev1.record()
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - w0)
            reps_ms.append(ev0.elapsed_time(ev1))
        ms = float(np.median(reps_ms))
        wall = float(np.median(walls))
        if not torch.isfinite(b).all():
            print("bench.py: non-finite field after the timed steps", file=sys.stderr)
            sys.exit(1)
        psteps = max(1, min(profile_steps, steps))
        (a, b), kms = wave.profile(a, b, psteps, **srcs(0, psteps))
        dom = max((k for k in kms if k in ALG_BYTES_PER_NODE), key=lambda k: kms[k])
        alg_bytes = ALG_BYTES_PER_NODE[dom] * esz * npts
        info = wave.info()
        # the dominant kernel's mean launch duration: a step of one launch (the one-pass
        # step) is timed by the events around the timed region (launches back to back);
        # a step of several launches by events around each launch (profile steps)
        single = info["kernels_per_step"] == 1 and len(kms) == 1
        kernel_ms = ms / steps if single else kms[dom]
        achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
        per_node = FUSED_STEP_BYTES_PER_NODE if info["fused_step"] else STEP_BYTES_PER_NODE
        step_gbps = per_node * esz * npts * steps / (ms / 1e3) / 1e9
        res = {"value": round(npts * steps / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms / steps, 5),
               "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                            "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                            "frac": round(achieved / HBM_PEAK_GBPS, 4),
                            "traffic": load_traffic(name, dom, alg_bytes),
                            "kernel_ms": round(kernel_ms, 5),
                            "timed_by": "timed region (one launch per step)" if single
                            else "events around each launch"},
               "step_algorithmic_bytes_per_node": per_node * esz,
               "step_algorithmic_GBps": round(step_gbps, 1),
               "step_frac_of_peak": round(step_gbps / HBM_PEAK_GBPS, 4),
               "kernel_ms": {k: round(v, 5) for k, v in kms.items()},
               "repeats_ms_per_step": [round(v / steps, 5) for v in reps_ms],
               "launch_plan": info, "wall_s_timed": round(wall, 4)}
        # HBM bytes the counters measured for every launch of a step (committed
        # rocprofv3 summary of the same sources), over the measured step time
        counted = [load_traffic(name, k, 0.0) for k in kms]
        if kms and all(c is not None for c in counted):
            per_step = sum(counted)
            gbps = per_step / (ms / steps / 1e3) / 1e9
            res["hbm_counted"] = {"bytes_per_step": round(per_step), "GBps": round(gbps, 1),
                                  "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4)}
        return a, b, res

    a, b, main = measure(a, b)
    two_pass = None
    if both and main["launch_plan"]["fused_step"]:
        wave.set_tuning(fused_step=False)
        a, b, two_pass = measure(a, b)
        two_pass.pop("launch_plan")
        wave.set_tuning(fused_step=True)
    wave.close()
    del a, b
    torch.cuda.empty_cache()
    return main, two_pass, create_ms


def f64_leg(adw, torch, steps: int, warmup: int, reps: int, profile_steps: int):
    """C3 at the paper's arithmetic: the same 8192^2 heterogeneous Ricker workload in
    FP64 (speed field and source rounded to FP64).  The handle's default step is the
    FP64 one-pass step on column strips (its truncation bound holds below 2^-53 at this
    r): 4E = 32 B per node and step algorithmically, HBM roofline 250,000 Mpts/s; the
    exact two-pass step beside it: 8E = 64 B, roofline 125,000 Mpts/s."""
    from paper_2006_10142_amd import workloads as wl
    name = "c3_heterogeneous_ricker_8192x8192_f64"
    prob = wl.config_c3(dtype="f64", nsteps=warmup + reps * steps)
    res, two_pass, create_ms = plain_leg(adw, torch, prob, name, "f64", steps, warmup, reps, profile_steps,
                                         both=True)
    one_pass = bool(res["launch_plan"]["fused_step"])
    res["workload"] = name
    res["dtype"] = "f64"
    res["steps"] = steps
    res["warmup"] = warmup
    res["create_ms"] = round(create_ms, 2)
    res["step"] = "one-pass" if one_pass else "two-pass"
    per_node = (FUSED_STEP_BYTES_PER_NODE if one_pass else STEP_BYTES_PER_NODE) * 8
    res["roofline_Mpts"] = round(HBM_PEAK_GBPS * 1e9 / per_node / 1e6, 1)
    res["launch_plan"] = {k: res["launch_plan"][k] for k in ("fused_step", "fused_tile_cols", "fused_tiles",
                                                             "fused_segment_rows", "fused_strips_wide")}
    if two_pass:
        two_pass["step"] = "two-pass"
        two_pass["roofline_Mpts"] = round(HBM_PEAK_GBPS * 1e9 / (STEP_BYTES_PER_NODE * 8) / 1e6, 1)
        res["two_pass"] = two_pass
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--reps", type=int, default=0,
                    help="timed repetitions of --steps steps; the median is reported "
                         "(default: at least 5, and at least 200 timed steps in all)")
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-cr", action="store_true", help="skip the cyclic-reduction baseline leg")
    ap.add_argument("--no-tridiag", action="store_true", help="skip the batched line-solve leg")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 leg of the workload")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one GPU; runs on several GPUs are not supported "
              "(--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2006_10142_amd as adw

    if args.reps <= 0:
        # the GPU's clocks move over the first tens of milliseconds of a run (the per-launch
        # durations dip and recover); enough repetitions put the median past that
        args.reps = max(5, -(-200 // max(1, args.steps)))
    name, dtype, n = WORKLOADS[args.workload]
    prob = make_problem(args.workload, args.warmup + args.reps * args.steps)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    main, two_pass, create_ms = plain_leg(adw, torch, prob, name, dtype, args.steps, args.warmup, args.reps,
                                          args.profile_steps, both=True)
    value = main["value"]
    # achievable copy bandwidth on this GPU (1 GiB read + 1 GiB write)
    x = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    adw.stream_copy(x, y)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        adw.stream_copy(x, y)
    c1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * x.numel() * 4 * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del x, y

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": name, "nx": prob.nx, "ny": prob.ny,
                   "coefficient": "per-node" if prob.c is not None else "constant",
                   "source": "ricker point source" if prob.src_amp is not None else "none",
                   "step": "one-pass" if main["launch_plan"]["fused_step"] else "two-pass",
                   "launch_plan": main["launch_plan"]},
        "roofline": main["roofline"],
        "step_algorithmic_bytes_per_node": main["step_algorithmic_bytes_per_node"],
        "step_algorithmic_GBps": main["step_algorithmic_GBps"],
        "step_frac_of_peak": main["step_frac_of_peak"],
        "hbm_counted": main.get("hbm_counted"),
        "kernel_ms": main["kernel_ms"],
        "repeats_ms_per_step": main["repeats_ms_per_step"],
        "reps": args.reps,
        "two_pass": two_pass,
        "copy_GBps": round(copy_gbps, 1),
        "create_ms": round(create_ms, 2),
        "wall_s_timed": main["wall_s_timed"],
    }
    for blk in (out, two_pass):
        hc = blk.get("hbm_counted") if blk else None
        if hc and copy_gbps > 0:
            hc["frac_of_copy"] = round(hc["GBps"] / copy_gbps, 4)
    tp_value = two_pass["value"] if two_pass else value
    if not args.no_f64 and args.workload == "c3":
        # the paper's arithmetic on the same workload: a short run (the FP64 step is
        # about twice as slow and its fields twice as large)
        out["f64"] = f64_leg(adw, torch, min(args.steps, 20), min(args.warmup, 5), args.reps,
                             min(args.profile_steps, 10))
    if not args.no_batch:
        out["batched"] = bench_batched(adw, torch, args.steps, args.warmup, value)
        out["batched"]["vs_two_pass"] = round(out["batched"]["value"] / tp_value, 4)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(adw, torch)
    if not args.no_tridiag:
        out["tridiag"] = bench_tridiag(adw, torch)
    if not args.no_cr and dtype == "f32":
        out["cr_baseline"] = bench_cr(adw, torch, prob, 10, value)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_steps)
    out["paper_context"] = PAPER_TABLE1
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
