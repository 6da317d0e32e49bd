"""Solver drivers above the C ABI (argument marshalling and host loops only).

* ``BatchState`` / ``solve_batched``: device state of one instance's R restarts and the fused
  persistent solver call (``fsmt_solve_batched``).
* ``PlainSolver``: the per-call path, a host loop of separate launches
  (cop_backward, pgd_step every step; round_and_check, erwa_update every level), one restart
  at a time; the reference point for the batched path's time-to-SAT.
* ``kappa_schedule``: the annealing schedule kappa_t = kmax t / (T ell) (sigma decreasing;
  Fig. 2 raises 1/sigma in equal increments), ell a length scale of the instance.
* ``COPObjective``: torch.autograd.Function returning U per restart, with the gradient from
  the reverse sweep (cop_backward).
"""
from __future__ import annotations

import ctypes as ct
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _abi
from . import (XBDD, cop_backward, cop_forward, erwa_update, fsmt_solve_batched, fsmt_solve_status,
               pgd_step, round_and_check)


def kappa_schedule(ell: float, levels: int = 40, kmax: float = 4.0) -> List[float]:
    return [kmax * t / levels / ell for t in range(1, levels + 1)]


@dataclass
class SolveConfig:
    kappas: Sequence[float]
    steps_per_level: int = 100
    eta_a: float = 0.5
    eta_b: float = 5.0
    eps: float = 1e-2
    rho: float = 0.5
    gamma: float = 2.0
    tau: int = 1
    normalize: bool = True
    stop_on_sat: int = 2
    schedule: int = 0        # 0 automatic, 1 persistent, 2 grid
    cluster: int = 0         # persistent schedule: workgroups per restart (0 automatic)
    level_begin: int = 0     # grid schedule: levels below this are complete for every restart
    spin_limit: int = 0      # cluster barrier polls before giving up (0: the library default)
    inst_schedule: Optional[Sequence[int]] = None   # per instance 0 (as schedule) / 1 / 2

    def abi(self):
        kap = (ct.c_double * max(1, len(self.kappas)))(*self.kappas)
        o = _abi.SolveOpts()
        o.kappas = ct.cast(kap, ct.c_void_p)
        o.n_levels = len(self.kappas)
        o.steps_per_level = int(self.steps_per_level)
        o.eta_a, o.eta_b, o.eps = float(self.eta_a), float(self.eta_b), float(self.eps)
        o.rho, o.gamma, o.tau = float(self.rho), float(self.gamma), int(self.tau)
        o.normalize = int(bool(self.normalize))
        o.stop_on_sat = int(self.stop_on_sat)
        o.schedule = int(self.schedule)
        o.cluster = int(self.cluster)
        o.level_begin = int(self.level_begin)
        o.spin_limit = int(self.spin_limit)
        keep = [kap]
        if self.inst_schedule is not None:
            sch = (ct.c_int32 * max(1, len(self.inst_schedule)))(*[int(v) for v in self.inst_schedule])
            o.inst_schedule = ct.cast(sch, ct.c_void_p)
            keep.append(sch)
        return o, keep


class BatchState:
    """Device tensors of one instance's R restarts (row-major [R][n])."""

    def __init__(self, h: XBDD, a0: np.ndarray, b0: np.ndarray, w0=None, device=None):
        import torch
        dev = device or torch.device("cuda", torch.cuda.current_device())
        R = a0.shape[0]
        self.h, self.R = h, R
        f32, i32 = torch.float32, torch.int32
        self.a = torch.as_tensor(np.ascontiguousarray(a0, np.float32), device=dev).reshape(R, h.n_bool)
        self.b = torch.as_tensor(np.ascontiguousarray(b0, np.float32), device=dev).reshape(R, h.n_real)
        if w0 is None:
            self.w = torch.ones(R, h.n_cons, dtype=f32, device=dev)
        else:
            self.w = torch.as_tensor(np.broadcast_to(w0, (R, h.n_cons)).astype(np.float32), device=dev).contiguous()
        self.hist = torch.zeros(R, h.n_cons, dtype=f32, device=dev)
        self.sat_bits = torch.zeros(R, max(1, (h.n_cons + 31) // 32), dtype=i32, device=dev)
        self.n_unsat = torch.full((R,), -1, dtype=i32, device=dev)
        self.verdict = torch.zeros(R, dtype=i32, device=dev)
        self.level_done = torch.zeros(R, dtype=i32, device=dev)
        self.steps_done = torch.zeros(R, dtype=i32, device=dev)
        self.obj = torch.zeros(R, dtype=f32, device=dev)

    def abi(self) -> _abi.SolveState:
        from . import view
        s = _abi.SolveState()
        s.a, s.b = view(self.a), view(self.b)
        for k in ("w", "hist", "sat_bits", "n_unsat", "verdict", "level_done", "steps_done", "obj"):
            setattr(s, k, getattr(self, k).data_ptr())
        s.grad_a = s.grad_b = None
        return s


def solve_batched(handles: Sequence[XBDD], states: Sequence[BatchState], cfg: SolveConfig, stream=None):
    """Enqueue one fused solver call (asynchronous; see ``check_batched``)."""
    o, keep = cfg.abi()
    fsmt_solve_batched(list(handles), o, [s.abi() for s in states], stream=stream)
    del keep


def check_batched(states: Sequence[BatchState], stream=None):
    """Wait for the stream and raise FsmtError (FSMT_EABORTED) if a solver call gave up."""
    fsmt_solve_status([s.abi() for s in states], stream=stream)


class PlainSolver:
    """Host loop of per-call launches for one instance and one restart (the plain
    per-instance path): a level's steps end when the step's gradient map norm is at most
    eps (Alg. "FourierSMT", per point)."""

    def __init__(self, h: XBDD, R: int = 1, device=None):
        import torch
        if R != 1:
            raise ValueError("the plain path runs one restart at a time")
        self.h, self.R = h, R
        dev = device or torch.device("cuda", torch.cuda.current_device())
        self.dev = dev
        self.ga = torch.zeros(R, h.n_bool, device=dev)
        self.gb = torch.zeros(R, h.n_real, device=dev)
        self.gsq = torch.zeros(R, device=dev)
        self.obj = torch.zeros(R, device=dev)
        nw = max(1, (h.n_cons + 31) // 32)
        self.bits = torch.zeros(R, nw, dtype=torch.int32, device=dev)
        self.nu = torch.zeros(R, dtype=torch.int32, device=dev)
        self.ver = torch.zeros(R, dtype=torch.int32, device=dev)

    def run(self, a0, b0, cfg: SolveConfig, stream=None):
        """Alg. CLS with Annealing for the R points of a0, b0; returns the trace summary.

        With a torch stream the host-side reads (gradient-map norm, verdict) are ordered
        after the launches on that stream.
        """
        import torch
        if isinstance(stream, torch.cuda.Stream):
            with torch.cuda.stream(stream):
                return self._run(a0, b0, cfg, stream)
        return self._run(a0, b0, cfg, stream)

    def _run(self, a0, b0, cfg: SolveConfig, stream=None):
        import torch
        h = self.h
        a = torch.as_tensor(np.ascontiguousarray(a0, np.float32), device=self.dev).reshape(self.R, h.n_bool).clone()
        b = torch.as_tensor(np.ascontiguousarray(b0, np.float32), device=self.dev).reshape(self.R, h.n_real).clone()
        w = torch.ones(self.R, h.n_cons, device=self.dev)
        hist = torch.zeros(self.R, h.n_cons, device=self.dev)
        self.ga.zero_()
        self.gb.zero_()
        steps = 0
        for t, kap in enumerate(cfg.kappas, start=1):
            for _ in range(cfg.steps_per_level):
                cop_backward(h, a, b, kap, w, None, self.ga, self.gb, flags=_abi.FSMT_ACCUMULATE, stream=stream)
                pgd_step(h, a, b, self.ga, self.gb, cfg.eta_a, cfg.eta_b, self.gsq, stream=stream)
                steps += 1
                if cfg.eps > 0 and float(self.gsq.max()) <= cfg.eps * cfg.eps:
                    break
            round_and_check(h, a, b, None, self.bits, self.nu, self.ver, stream=stream)
            erwa_update(h, self.R, self.bits, w, hist, t, cfg.rho, cfg.gamma, cfg.tau, cfg.normalize,
                        stream=stream)
            if int(self.ver.max()) == 1:
                return dict(verdict=1, level=t, steps=steps, a=a, b=b)
        return dict(verdict=0, level=len(cfg.kappas), steps=steps, a=a, b=b)


def _autograd():
    import torch

    class COPObjective(torch.autograd.Function):
        """U(a, b) per restart; backward uses the reverse sweep of cop_backward.

        forward(a [R][n], b [R][m], handle, kappa, w [C] or [R][C]) -> U [R]. The gradient
        is computed in the same launch as U when a or b requires grad, and scaled by the
        incoming gradient in backward (no node messages are stored).
        """

        @staticmethod
        def forward(ctx, a, b, handle, kappa, w):
            R = a.shape[0]
            obj = torch.zeros(R, device=a.device)
            need = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
            if need:
                # variable-major [n][R] storage viewed as [R][n]: the restarts of one
                # constraint update consecutive words, so the gradient atomics coalesce
                ga = torch.zeros(a.shape[1], a.shape[0], device=a.device).t()
                gb = torch.zeros(b.shape[1], b.shape[0], device=b.device).t()
                cop_backward(handle, a.detach(), b.detach(), kappa, w, obj, ga, gb)
                ctx.save_for_backward(ga, gb)
            else:
                cop_forward(handle, a.detach(), b.detach(), kappa, w, obj)
            return obj

        @staticmethod
        def backward(ctx, g):
            ga, gb = ctx.saved_tensors
            return g[:, None] * ga, g[:, None] * gb, None, None, None

    return COPObjective


def cop_objective(a, b, handle: XBDD, kappa: float, w):
    """Differentiable U per restart (torch.autograd)."""
    return _autograd().apply(a, b, handle, kappa, w)


def time_to_sat_batched(handles, states, cfg: SolveConfig, stream=None):
    """Wall time of one fused launch (compile and upload excluded) and the verdicts."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solve_batched(handles, states, cfg, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    check_batched(states, stream=stream)
    return dt


__all__ = ["kappa_schedule", "SolveConfig", "BatchState", "solve_batched", "check_batched", "PlainSolver",
           "cop_objective", "time_to_sat_batched", "Optional"]
