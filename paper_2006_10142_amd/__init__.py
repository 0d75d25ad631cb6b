"""MI355X (gfx950) ADI solver for the implicit finite-difference 2-D acoustic
wave equation (Altybay, Ruzhansky, Tokmagambetov, Sec. 2 scheme, Sec. 3 time loop).

Thin Python binding of libadiwave.so: argument marshalling only.  Every
arithmetic step runs in the HIP kernels; PyTorch supplies device memory and the
current stream.  There is no CPU fallback: a missing library raises.

    import torch, paper_2006_10142_amd as adw
    wave = adw.Wave(nx, ny, h, dt, c=speed_tensor_or_scalar, dtype=torch.float32)
    u1 = wave.start(u0, mode="ghost")
    u_prev, u_curr = wave.step(u0, u1, nsteps=100)
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

from . import _lib
from ._lib import AdiError

__all__ = ["Wave", "Batch", "ADIWaveFunction", "simulate_traces", "tridiag_solve_batched",
           "stream_copy", "AdiError", "lib_path"]

lib_path = _lib.LIB_PATH


def _torch():
    import torch
    return torch


def _dtype_code(dtype) -> int:
    torch = _torch()
    if dtype == torch.float32:
        return _lib.ADI_F32
    if dtype == torch.float64:
        return _lib.ADI_F64
    raise TypeError(f"unsupported dtype {dtype} (float32 or float64)")


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _field(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _index(t, name):
    torch = _torch()
    if t.device.type != "cuda" or t.dtype != torch.int32 or not t.is_contiguous() or t.dim() != 1:
        raise ValueError(f"{name} must be a contiguous 1-D int32 device tensor")
    return t


class Wave:
    """Handle of one nx x ny grid (interior nodes, spacing h, time step dt).

    c: wave speed, scalar or (ny, nx) device tensor; the coefficient of the
    Laplacian is kappa = c**2.  Alternatively pass ``kappa=`` directly.
    """

    def __init__(self, nx: int, ny: int, h: float, dt: float, c=1.0, dtype=None,
                 kappa=None):
        torch = _torch()
        dtype = torch.float32 if dtype is None else dtype
        self.nx, self.ny, self.h, self.dt, self.dtype = int(nx), int(ny), float(h), float(dt), dtype
        self._code = _dtype_code(dtype)
        lib = _lib.load()
        handle = ctypes.c_void_p()
        speed_ptr, speed_scalar = None, 1.0
        if kappa is None and isinstance(c, torch.Tensor):
            speed_ptr = _field(c, dtype, (self.ny, self.nx), "c")
        elif kappa is None:
            speed_scalar = float(c)
        self._stream = torch.cuda.current_stream().cuda_stream
        _lib.check(lib.adi_wave_create(ctypes.byref(handle), self.nx, self.ny, self.h, self.dt,
                                       speed_ptr, speed_scalar, self._code,
                                       ctypes.c_void_p(self._stream)))
        self._h = handle
        if kappa is not None:
            self.set_kappa(kappa)

    # -- plumbing ------------------------------------------------------------
    def _sync_stream(self):
        s = _torch().cuda.current_stream().cuda_stream
        if s != self._stream:
            _lib.check(_lib.load().adi_wave_set_stream(self._h, ctypes.c_void_p(s)))
            self._stream = s

    def _shape(self):
        return (self.ny, self.nx)

    def _sources(self, src_idx, src_amp, nsteps):
        if src_idx is None or src_idx.numel() == 0:
            return None
        _index(src_idx, "src_idx")
        n = src_idx.numel()
        if src_amp is None or src_amp.dtype != self.dtype or src_amp.device.type != "cuda" \
                or not src_amp.is_contiguous() or src_amp.numel() < nsteps * n:
            raise ValueError("src_amp must be a contiguous device tensor of the handle dtype "
                             "holding nsteps x count values")
        return _lib.AdiSource(n, src_idx.data_ptr(), src_amp.data_ptr())

    # -- API -----------------------------------------------------------------
    def set_kappa(self, kappa):
        """Replace the coefficient by kappa (scalar or (ny, nx) device tensor)."""
        self._sync_stream()
        torch = _torch()
        if isinstance(kappa, torch.Tensor):
            ptr, sc = _field(kappa, self.dtype, self._shape(), "kappa"), 1.0
        else:
            ptr, sc = None, float(kappa)
        _lib.check(_lib.load().adi_wave_set_kappa(self._h, ptr, sc))

    def start(self, u0, psi=None, src_idx=None, src_amp0=None, mode: str = "ghost", out=None):
        """Level u^1 from u^0 (mode 'paper': eq. (CN2); 'ghost': second-order start)."""
        self._sync_stream()
        torch = _torch()
        p0 = _field(u0, self.dtype, self._shape(), "u0")
        pp = None if psi is None else _field(psi, self.dtype, self._shape(), "psi")
        u1 = torch.empty_like(u0) if out is None else out
        p1 = _field(u1, self.dtype, self._shape(), "u1")
        src = self._sources(src_idx, src_amp0, 1)
        m = {"paper": _lib.ADI_START_PAPER, "ghost": _lib.ADI_START_GHOST}[mode]
        _lib.check(_lib.load().adi_wave_start(self._h, p0, pp,
                                              ctypes.byref(src) if src else None, m, p1))
        return u1

    def step(self, u_prev, u_curr, nsteps: int = 1, src_idx=None, src_amp=None,
             rec_idx=None, traces=None) -> Tuple:
        """nsteps ADI steps; returns (u_prev, u_curr) holding u^{n+nsteps-1}, u^{n+nsteps}.

        The two tensors are reused: u^{n+1} overwrites u^{n-1} each step, so the
        returned pair is (u_prev, u_curr) or (u_curr, u_prev) depending on parity.
        rec_idx/traces: int32 node offsets and a (nsteps, count) output tensor.
        """
        self._sync_stream()
        a = _field(u_prev, self.dtype, self._shape(), "u_prev")
        b = _field(u_curr, self.dtype, self._shape(), "u_curr")
        src = self._sources(src_idx, src_amp, nsteps)
        rec = None
        if rec_idx is not None and rec_idx.numel() > 0:
            _index(rec_idx, "rec_idx")
            if traces is None or traces.dtype != self.dtype or not traces.is_contiguous() \
                    or traces.numel() < nsteps * rec_idx.numel():
                raise ValueError("traces must be a contiguous (nsteps, count) tensor of the handle dtype")
            rec = _lib.AdiReceivers(rec_idx.numel(), rec_idx.data_ptr(), traces.data_ptr())
        pa, pb = ctypes.c_void_p(a.value), ctypes.c_void_p(b.value)
        _lib.check(_lib.load().adi_wave_step(self._h, ctypes.byref(pa), ctypes.byref(pb),
                                             ctypes.byref(src) if src else None,
                                             ctypes.byref(rec) if rec else None, int(nsteps)))
        if pb.value == b.value:
            return u_prev, u_curr
        return u_curr, u_prev

    def step_tdc(self, u_prev, u_curr, kappa_prev=None, kappa_next=None, src_idx=None, src_amp=None,
                 rec_idx=None, traces=None) -> Tuple:
        """One step of eq. (CN1) with a time-dependent coefficient: kappa_prev multiplies the
        Laplacian of u^{n-1}, kappa_next that of u^{n+1} ((ny, nx) device tensors; None =
        the current coefficient).  kappa_next becomes the handle's coefficient.  Returns
        (u_prev, u_curr) rotated as by step(..., 1)."""
        self._sync_stream()
        a = _field(u_prev, self.dtype, self._shape(), "u_prev")
        b = _field(u_curr, self.dtype, self._shape(), "u_curr")
        kp = None if kappa_prev is None else _field(kappa_prev, self.dtype, self._shape(), "kappa_prev")
        kn = None if kappa_next is None else _field(kappa_next, self.dtype, self._shape(), "kappa_next")
        src = self._sources(src_idx, src_amp, 1)
        rec = None
        if rec_idx is not None and rec_idx.numel() > 0:
            _index(rec_idx, "rec_idx")
            if traces is None or traces.dtype != self.dtype or not traces.is_contiguous() \
                    or traces.numel() < rec_idx.numel():
                raise ValueError("traces must be a contiguous tensor of the handle dtype with count values")
            rec = _lib.AdiReceivers(rec_idx.numel(), rec_idx.data_ptr(), traces.data_ptr())
        pa, pb = ctypes.c_void_p(a.value), ctypes.c_void_p(b.value)
        _lib.check(_lib.load().adi_wave_step_tdc(self._h, ctypes.byref(pa), ctypes.byref(pb), kp, kn,
                                                 ctypes.byref(src) if src else None,
                                                 ctypes.byref(rec) if rec else None))
        if pb.value == b.value:
            return u_prev, u_curr
        return u_curr, u_prev

    SPLIT_MODES = {"fr": 1, "theta1": 2}

    def step_split(self, u_half, u_curr, mode="fr", src_idx=None, src_amp=None, src_amp_half=None,
                   rec_idx=None, traces=None) -> Tuple:
        """One pair of sub-steps of the split as printed (mode "fr": eqs. (fr1)-(fr2);
        "theta1": Listing 1's line systems).  u_half holds u^{k-1/2} and becomes
        u^{k+1/2}; u_curr holds u^k and becomes u^{k+1} (in place).  src_amp: values
        of f^k at src_idx, src_amp_half: of f^{k+1/2}; traces: receivers of u^{k+1}."""
        self._sync_stream()
        a = _field(u_half, self.dtype, self._shape(), "u_half")
        b = _field(u_curr, self.dtype, self._shape(), "u_curr")
        src = self._sources(src_idx, src_amp, 1) if src_amp is not None else None
        src_h = self._sources(src_idx, src_amp_half, 1) if src_amp_half is not None else None
        rec = None
        if rec_idx is not None and rec_idx.numel() > 0:
            _index(rec_idx, "rec_idx")
            if traces is None or traces.dtype != self.dtype or not traces.is_contiguous() \
                    or traces.numel() < rec_idx.numel():
                raise ValueError("traces must be a contiguous tensor of the handle dtype with count values")
            rec = _lib.AdiReceivers(rec_idx.numel(), rec_idx.data_ptr(), traces.data_ptr())
        _lib.check(_lib.load().adi_wave_step_split(self._h, self.SPLIT_MODES[mode], a, b,
                                                   ctypes.byref(src) if src else None,
                                                   ctypes.byref(src_h) if src_h else None,
                                                   ctypes.byref(rec) if rec else None))
        return u_half, u_curr

    def profile(self, u_prev, u_curr, nsteps: int, src_idx=None, src_amp=None):
        """Run nsteps steps with per-launch events; returns ((u_prev, u_curr), {kernel: mean ms})."""
        self._sync_stream()
        a = _field(u_prev, self.dtype, self._shape(), "u_prev")
        b = _field(u_curr, self.dtype, self._shape(), "u_curr")
        src = self._sources(src_idx, src_amp, nsteps)
        ms = (ctypes.c_double * 8)()
        names = (ctypes.c_char_p * 8)()
        nk = ctypes.c_int(0)
        pa, pb = ctypes.c_void_p(a.value), ctypes.c_void_p(b.value)
        _lib.check(_lib.load().adi_wave_profile(self._h, ctypes.byref(pa), ctypes.byref(pb),
                                                ctypes.byref(src) if src else None, int(nsteps),
                                                ms, names, ctypes.byref(nk)))
        out = {names[k].decode(): ms[k] for k in range(nk.value)}
        levels = (u_prev, u_curr) if pb.value == b.value else (u_curr, u_prev)
        return levels, out

    def _receivers(self, rec_idx, traces, nsteps):
        if rec_idx is None or rec_idx.numel() == 0:
            return None
        _index(rec_idx, "rec_idx")
        if traces is None or traces.dtype != self.dtype or not traces.is_contiguous() \
                or traces.numel() < nsteps * rec_idx.numel():
            raise ValueError("traces must be a contiguous (nsteps, count) tensor of the handle dtype")
        return _lib.AdiReceivers(rec_idx.numel(), rec_idx.data_ptr(), traces.data_ptr())

    def adjoint_forward(self, u_prev, u_curr, nsteps: int, src_idx=None, src_amp=None,
                        rec_idx=None, checkpoint_every: int = 100):
        """Forward run keeping checkpoints for adjoint_backward; returns the traces
        (nsteps, nrec) (u_prev and u_curr are not modified)."""
        torch = _torch()
        self._sync_stream()
        a = _field(u_prev, self.dtype, self._shape(), "u_prev")
        b = _field(u_curr, self.dtype, self._shape(), "u_curr")
        src = self._sources(src_idx, src_amp, nsteps)
        nrec = 0 if rec_idx is None else rec_idx.numel()
        traces = torch.zeros((nsteps, nrec), dtype=self.dtype, device=u_curr.device)
        rec = self._receivers(rec_idx, traces, nsteps)
        rid = ctypes.c_ulonglong(0)
        _lib.check(_lib.load().adi_adjoint_forward(self._h, a, b, ctypes.byref(src) if src else None,
                                                   ctypes.byref(rec) if rec else None, int(nsteps),
                                                   int(checkpoint_every), ctypes.byref(rid)))
        self._adj_steps = int(nsteps)
        self.adjoint_record = int(rid.value)
        return traces

    def adjoint_backward(self, grad_traces, src_idx=None, src_amp=None, rec_idx=None,
                         want_amp: bool = False, record: int = 0):
        """Reverse pass of the stored forward run: returns (dJ/dkappa, dJ/d source values or None).
        record: the id adjoint_forward left in self.adjoint_record (0: the stored run);
        raises AdiError when that run was replaced or the coefficient changed since."""
        torch = _torch()
        self._sync_stream()
        nsteps = self._adj_steps
        src = self._sources(src_idx, src_amp, nsteps)
        gt = grad_traces.contiguous().to(self.dtype)
        rec = self._receivers(rec_idx, gt, nsteps)
        gk = torch.empty(self._shape(), dtype=self.dtype, device=gt.device)
        ga = None
        if want_amp and src is not None:
            ga = torch.zeros((nsteps, src_idx.numel()), dtype=self.dtype, device=gt.device)
        _lib.check(_lib.load().adi_adjoint_backward(
            self._h, ctypes.c_ulonglong(int(record)), ctypes.byref(src) if src else None,
            ctypes.byref(rec) if rec else None,
            ctypes.c_void_p(gt.data_ptr()), ctypes.c_void_p(gk.data_ptr()),
            None if ga is None else ctypes.c_void_p(ga.data_ptr())))
        return gk, ga

    def info(self) -> dict:
        inf = _lib.AdiWaveInfo()
        _lib.check(_lib.load().adi_wave_get_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _lib.AdiWaveInfo._fields_}

    def set_tuning(self, x_threads_per_line=0, x_rows_per_strip=0, y_fused=None,
                   y_chunk_rows=0, fused_step=None, cyclic_reduction=None, fused_tile_cols=0,
                   fused_lane_nodes=0, fused_segment_rows=0):
        """Override the launch plan (0 / None keeps the current value).  fused_step:
        True = one-pass step (when its truncation bound holds: FP32 r <= 0.18 and nx % 4
        == 0, FP64 r <= 0.13 and nx even), False = exact two-pass step.  cyclic_reduction: True = the paper's cyclic-reduction line
        solver (one launch per level, for comparison), False = the default solvers.
        fused_tile_cols: one-pass tile width (multiple of 8, <= 496; FP64 strips <= 64;
        -1 = automatic).
        fused_lane_nodes: one-pass x-line nodes per lane, 8 or 4 (4: tiles of at most
        240 columns that keep r in LDS for the y-lines).  fused_segment_rows: one-pass
        step on column strips (<= 240 columns), each workgroup marching down this many output rows (>= 8);
        -2 = 64-row tiles, -1 = automatic."""
        self._sync_stream()
        f = 0 if y_fused is None else (1 if y_fused else 2)
        fs = 0 if fused_step is None else (1 if fused_step else 2)
        ls = 0 if cyclic_reduction is None else (2 if cyclic_reduction else 1)
        t = _lib.AdiTuning(x_threads_per_line, x_rows_per_strip, f, y_chunk_rows, fs, ls,
                           fused_tile_cols, fused_lane_nodes, fused_segment_rows)
        _lib.check(_lib.load().adi_wave_set_tuning(self._h, ctypes.byref(t)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.load().adi_wave_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent simulations of uneven grid sizes advanced together.

    sizes: list of (nx, ny); h, dt: per-simulation lists; c: per-simulation
    speed (scalar or (ny, nx) device tensor).  One launch per kernel covers the
    whole batch each step; optionally captured in a hipGraph.
    """

    def __init__(self, sizes, h, dt, c, dtype=None):
        torch = _torch()
        dtype = torch.float32 if dtype is None else dtype
        self.dtype = dtype
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        n = len(self.sizes)
        if not (len(h) == len(dt) == len(c) == n):
            raise ValueError("sizes, h, dt and c must have one entry per simulation")
        self.count = n
        self._code = _dtype_code(dtype)
        nxa = (ctypes.c_int * n)(*[s[0] for s in self.sizes])
        nya = (ctypes.c_int * n)(*[s[1] for s in self.sizes])
        ha = (ctypes.c_double * n)(*[float(v) for v in h])
        dta = (ctypes.c_double * n)(*[float(v) for v in dt])
        sp = (ctypes.c_void_p * n)()
        sc = (ctypes.c_double * n)()
        self._keep = []
        for k, ck in enumerate(c):
            if isinstance(ck, torch.Tensor):
                sp[k] = _field(ck, dtype, (self.sizes[k][1], self.sizes[k][0]), f"c[{k}]").value
                sc[k] = 1.0
                self._keep.append(ck)
            else:
                sp[k] = None
                sc[k] = float(ck)
        self._stream = torch.cuda.current_stream().cuda_stream
        handle = ctypes.c_void_p()
        _lib.check(_lib.load().adi_batch_create(ctypes.byref(handle), n, nxa, nya, ha, dta, sp, sc,
                                                self._code, ctypes.c_void_p(self._stream)))
        self._h = handle
        self._levels = None

    def bind(self, u_prev, u_curr):
        """Bind the two levels of every simulation (lists of (ny, nx) device tensors)."""
        n = self.count
        a = (ctypes.c_void_p * n)()
        b = (ctypes.c_void_p * n)()
        for k in range(n):
            shp = (self.sizes[k][1], self.sizes[k][0])
            a[k] = _field(u_prev[k], self.dtype, shp, f"u_prev[{k}]").value
            b[k] = _field(u_curr[k], self.dtype, shp, f"u_curr[{k}]").value
        _lib.check(_lib.load().adi_batch_bind(self._h, a, b))
        self._levels = {t.data_ptr(): t for t in list(u_prev) + list(u_curr)}

    def start(self, mode: str = "ghost"):
        m = {"paper": _lib.ADI_START_PAPER, "ghost": _lib.ADI_START_GHOST}[mode]
        _lib.check(_lib.load().adi_batch_start(self._h, m))

    def step(self, nsteps: int = 1):
        _lib.check(_lib.load().adi_batch_step(self._h, int(nsteps)))

    def levels(self):
        """(u_prev list, u_curr list) as the bound tensors, in their current roles."""
        n = self.count
        a = (ctypes.c_void_p * n)()
        b = (ctypes.c_void_p * n)()
        _lib.check(_lib.load().adi_batch_levels(self._h, a, b))
        return [self._levels[a[k]] for k in range(n)], [self._levels[b[k]] for k in range(n)]

    def graph(self, enable: bool = True):
        _lib.check(_lib.load().adi_batch_graph(self._h, 1 if enable else 0))

    def plan(self) -> dict:
        p = _lib.AdiBatchPlan()
        _lib.check(_lib.load().adi_batch_get_plan(self._h, ctypes.byref(p)))
        return {f: getattr(p, f) for f, _ in _lib.AdiBatchPlan._fields_}

    def set_plan(self, x_threads_per_line=0, x_grid=0, yscan_grid=0, ysolve_grid=0, fused_step=None,
                 fused_lane_nodes=0, fused_strips=None):
        """Launch plan of the two-pass step; fused_step: True = one-pass step for every
        simulation (FP32, when allowed), False = exact two-pass step, None = keep;
        fused_lane_nodes: 8 or 4 nodes per lane of the one-pass tiles (0 = keep);
        fused_strips: True = the one-pass step on column strips, False = on tiles,
        None = keep."""
        p = _lib.AdiBatchPlan()
        _lib.check(_lib.load().adi_batch_get_plan(self._h, ctypes.byref(p)))
        if x_threads_per_line:
            p.x_threads_per_line = x_threads_per_line
        p.x_grid, p.yscan_grid, p.ysolve_grid = x_grid, yscan_grid, ysolve_grid
        p.fused_step = 0 if fused_step is None else (1 if fused_step else 2)
        p.fused_lane_nodes = fused_lane_nodes
        p.fused_strips = 0 if fused_strips is None else (1 if fused_strips else 2)
        _lib.check(_lib.load().adi_batch_set_plan(self._h, ctypes.byref(p)))

    def autotune(self, trial_steps: int = 10, cache: Optional[str] = None) -> float:
        """Pick the fastest plan (or reuse one cached in the JSON file `cache`)."""
        import json
        import os
        key = None
        if cache:
            import hashlib
            key = hashlib.sha256(repr((self._code, self.sizes)).encode()).hexdigest()[:20]
            if os.path.exists(cache):
                try:
                    ent = json.load(open(cache)).get(key)
                except Exception:
                    ent = None
                if ent:
                    strips = ent.get("fused_strips")
                    self.set_plan(ent["x_threads_per_line"], ent["x_grid"], ent["yscan_grid"],
                                  ent["ysolve_grid"], fused_lane_nodes=ent.get("fused_lane_nodes", 0),
                                  fused_strips=None if strips is None else bool(strips))
                    return float(ent["ms_per_step"])
        best = ctypes.c_double(0.0)
        _lib.check(_lib.load().adi_batch_autotune(self._h, int(trial_steps), ctypes.byref(best)))
        if cache:
            p = self.plan()
            data = {}
            if os.path.exists(cache):
                try:
                    data = json.load(open(cache))
                except Exception:
                    data = {}
            data[key] = {k: p[k] for k in ("x_threads_per_line", "x_grid", "yscan_grid",
                                           "ysolve_grid", "fused_lane_nodes", "fused_strips")}
            data[key]["ms_per_step"] = best.value
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            json.dump(data, open(cache, "w"), indent=1)
        return best.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.load().adi_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ADIWaveFunction:
    """torch.autograd.Function: traces = ADIWaveFunction.apply(kappa, src_amp, wave, u_prev,
    u_curr, nsteps, src_idx, rec_idx, checkpoint_every).

    Forward: set the handle's coefficient to kappa, run nsteps steps with
    checkpoints, return the receiver traces (nsteps, nrec).  Backward: the
    adjoint reverse pass gives dJ/dkappa (and dJ/d src_amp).  One forward per
    handle may be pending a backward at a time: a second forward on the same
    handle (or a coefficient change) before the first backward makes that
    backward raise AdiError instead of returning another run's gradient.
    """
    _fn = None

    @classmethod
    def apply(cls, *args):
        return cls._function().apply(*args)

    @classmethod
    def _function(cls):
        if cls._fn is None:
            torch = _torch()

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, kappa, src_amp, wave, u_prev, u_curr, nsteps, src_idx, rec_idx,
                            checkpoint_every):
                    wave.set_kappa(kappa.detach().contiguous())
                    amp = None if src_amp is None else src_amp.detach().contiguous()
                    tr = wave.adjoint_forward(u_prev, u_curr, nsteps, src_idx=src_idx, src_amp=amp,
                                              rec_idx=rec_idx, checkpoint_every=checkpoint_every)
                    ctx.wave, ctx.src_idx, ctx.rec_idx, ctx.amp = wave, src_idx, rec_idx, amp
                    ctx.record = wave.adjoint_record
                    return tr

                @staticmethod
                def backward(ctx, grad_traces):
                    want_amp = ctx.amp is not None and ctx.needs_input_grad[1]
                    gk, ga = ctx.wave.adjoint_backward(grad_traces, src_idx=ctx.src_idx,
                                                       src_amp=ctx.amp, rec_idx=ctx.rec_idx,
                                                       want_amp=want_amp, record=ctx.record)
                    return gk, ga, None, None, None, None, None, None, None

            cls._fn = _F
        return cls._fn


def simulate_traces(wave, kappa, u_prev, u_curr, nsteps, src_idx, src_amp, rec_idx,
                    checkpoint_every: int = 100):
    """Differentiable receiver traces of a run (see ADIWaveFunction)."""
    return ADIWaveFunction.apply(kappa, src_amp, wave, u_prev, u_curr, nsteps, src_idx, rec_idx,
                                 checkpoint_every)


def tridiag_solve_batched(a, b, c, d, n: int, batch: int, sys_stride: int, elem_stride: int = 1,
                          noalloc: bool = False):
    """Solve batch tridiagonal systems in place in d (see tridiag_solve_batched in adiwave.h).
    noalloc=True calls tridiag_solve_batched_noalloc: no device allocation, the library's
    fixed 64 MiB scratch instead (larger workspaces raise)."""
    torch = _torch()
    for name, t in (("a", a), ("b", b), ("c", c), ("d", d)):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous device tensor")
        if t.dtype != d.dtype:
            raise TypeError("a, b, c and d must share one dtype")
    if n > 0 and batch > 0:
        need = (batch - 1) * sys_stride + (n - 1) * elem_stride + 1
        for name, t in (("a", a), ("b", b), ("c", c), ("d", d)):
            if t.numel() < need:
                raise ValueError(f"{name} holds {t.numel()} values, the layout needs {need}")
    code = _dtype_code(d.dtype)
    fn = _lib.load().tridiag_solve_batched_noalloc if noalloc else _lib.load().tridiag_solve_batched
    _lib.check(fn(code, int(n), int(batch), a.data_ptr(), b.data_ptr(), c.data_ptr(), d.data_ptr(),
                  int(sys_stride), int(elem_stride), _stream_ptr()))
    return d


def stream_copy(src, dst):
    """Device copy through the library's plain copy kernel (bandwidth reference)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst too small")
    _lib.check(_lib.load().adi_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream_ptr()))
    return dst
