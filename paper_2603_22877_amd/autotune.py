"""Measured plan selection for the batched solver (fsmt_solve_batched).

The library picks a schedule per instance from a cost model (persistent: one workgroup
cluster per restart with the state in LDS; grid: one captured graph of grid-wide kernels per
level) and a cluster size from an occupancy query. The tuner replaces the model by
measurement: every candidate plan runs a short fixed-work launch of the caller's own batch
(one level of ``steps`` and of ``2 steps`` projected-gradient iterations, so the per-iteration
cost and the level-end cost separate), scored as one level of the caller's configuration.
Candidates: the model's plan; every instance persistent with the automatic cluster and with
each cluster size the device can hold; every instance on the grid; and, for a batch, the
per-instance choice of the faster schedule measured on each instance alone. The winner is
cached on disk, keyed by the device, the library build and a signature of the instances
(sizes, diagram statistics, restarts), so a later call with the same shapes reuses it.

Argument marshalling and timing only: every candidate runs the library's kernels.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import _abi, xbdd_info
from .solver import BatchState, SolveConfig, solve_batched

CACHE_ENV = "FSMT_TUNE_CACHE"


@dataclass
class Plan:
    inst_schedule: List[int]          # per instance: 1 persistent, 2 grid, 0 the model's choice
    cluster: int = 0                  # persistent schedule: workgroups per restart (0 automatic)
    label: str = "model"
    us_per_level: float = 0.0         # measured: one level of the caller's configuration
    us_per_step: float = 0.0          # measured: one projected-gradient iteration
    candidates: Dict[str, float] = field(default_factory=dict)   # label -> us per level
    cached: bool = False

    def apply(self, cfg: SolveConfig) -> SolveConfig:
        return dataclasses.replace(cfg, schedule=0, inst_schedule=list(self.inst_schedule), cluster=self.cluster)

    def as_dict(self) -> dict:
        return {"label": self.label, "inst_schedule": self.inst_schedule, "cluster": self.cluster,
                "us_per_level": self.us_per_level, "us_per_step": self.us_per_step,
                "candidates": self.candidates, "cached": self.cached}


def _cache_path() -> str:
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "fsmt_autotune.json"))


def signature(handles, restarts: Sequence[int], cfg: SolveConfig) -> str:
    """Device, library build and instance shapes: what the measured times depend on."""
    import torch
    lib = _abi.LIB_PATH
    st = os.stat(lib)
    parts = [torch.cuda.get_device_name(), f"{st.st_size}:{int(st.st_mtime)}", f"steps={cfg.steps_per_level}"]
    for h, R in zip(handles, restarts):
        i = xbdd_info(h)
        parts.append(",".join(str(i[k]) for k in ("n_cons", "n_bool", "n_real", "n_templates", "max_nodes",
                                                   "max_slots", "n_gd", "n_pair", "n_big", "n_halfspaces",
                                                   "hs_separable", "table_bytes")) + f",R={R}")
    return hashlib.sha256("|".join(parts).encode()).hexdigest()[:32]


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(key: str, plan: Plan) -> None:
    path = _cache_path()
    data = _load_cache()
    data[key] = plan.as_dict()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f)
        os.replace(tmp, path)
    except OSError:
        pass


def _time_launch(handles, init, cfg: SolveConfig, steps: int, reps: int, stream) -> float:
    """Best of ``reps`` launches of one level of ``steps`` iterations (ms, HIP events)."""
    import torch
    c = dataclasses.replace(cfg, kappas=list(cfg.kappas[:1]), steps_per_level=steps, eps=0.0, stop_on_sat=0,
                            level_begin=0)
    best = float("inf")
    for _ in range(reps):
        states = [BatchState(h, a, b) for h, (a, b) in zip(handles, init)]
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solve_batched(handles, states, c, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def measure(handles, init, cfg: SolveConfig, steps: int = 8, reps: int = 2, stream=None) -> Tuple[float, float]:
    """(us per iteration, us per level of cfg.steps_per_level iterations) of cfg's plan."""
    import torch
    stream = stream or torch.cuda.current_stream()
    t1 = _time_launch(handles, init, cfg, steps, reps, stream)
    t2 = _time_launch(handles, init, cfg, 2 * steps, reps, stream)
    it = max(t2 - t1, 1e-6) / steps
    level_end = max(t1 - steps * it, 0.0)
    return it * 1e3, (cfg.steps_per_level * it + level_end) * 1e3


def cached_plan(handles, init: Sequence[Tuple], cfg: SolveConfig) -> Optional[Plan]:
    """The cached plan for this batch and configuration, or None (nothing is measured)."""
    hit = _load_cache().get(signature(handles, [a.shape[0] for a, _ in init], cfg))
    if hit is None:
        return None
    return Plan(inst_schedule=list(hit["inst_schedule"]), cluster=int(hit["cluster"]), label=hit["label"],
                us_per_level=hit["us_per_level"], us_per_step=hit["us_per_step"],
                candidates=dict(hit["candidates"]), cached=True)


def tune(handles, init: Sequence[Tuple], cfg: SolveConfig, steps: int = 16, reps: int = 3, use_cache: bool = True,
         stream=None, log: Optional[Callable[[str], None]] = None, margin: float = 0.03) -> Plan:
    """Measure the candidate plans for this batch (handles with their initial points ``init``,
    one (a0, b0) pair per instance) under ``cfg`` and return the fastest. The model's plan is
    kept unless another is faster by more than ``margin`` (the per-level estimate extrapolates
    a difference of two short launches, so plans that run the same kernels differ by noise)."""
    import torch
    stream = stream or torch.cuda.Stream()
    restarts = [a.shape[0] for a, _ in init]
    n = len(handles)
    key = signature(handles, restarts, cfg)
    if use_cache:
        hit = cached_plan(handles, init, cfg)
        if hit is not None:
            return hit

    results: Dict[str, Tuple[float, float, Plan]] = {}

    def trial(plan: Plan) -> None:
        try:
            it, lvl = measure(handles, init, plan.apply(cfg), steps, reps, stream)
        except _abi.FsmtError as e:   # a plan the device cannot run (LDS, co-residency)
            if log:
                log(f"autotune: {plan.label} not runnable ({e})")
            return
        results[plan.label] = (it, lvl, plan)
        if log:
            log(f"autotune: {plan.label}: {it:.1f} us per iteration, {lvl / 1e3:.2f} ms per level")

    trial(Plan([0] * n, 0, "model"))
    trial(Plan([1] * n, 0, "persistent"))
    for k in (1, 2, 4, 8, 16):
        trial(Plan([1] * n, k, f"persistent k={k}"))
    trial(Plan([2] * n, 0, "grid"))
    if n > 1:
        # per instance: the faster schedule of the instance alone, then the combination
        choice = []
        for i in range(n):
            one_h, one_i = [handles[i]], [init[i]]
            best, pick = float("inf"), 0
            for sched in (1, 2):
                c = dataclasses.replace(cfg, schedule=sched, inst_schedule=None, cluster=0)
                try:
                    _, lvl = measure(one_h, one_i, c, steps, 1, stream)
                except _abi.FsmtError:
                    continue
                if lvl < best:
                    best, pick = lvl, sched
            choice.append(pick)
        trial(Plan(choice, 0, "per-instance"))
    if not results:
        raise RuntimeError("autotune: no candidate plan could run")
    label = min(results, key=lambda k: results[k][1])
    if "model" in results and results["model"][1] <= (1.0 + margin) * results[label][1]:
        label = "model"
    it, lvl, plan = results[label]
    plan.us_per_step, plan.us_per_level = it, lvl
    plan.candidates = {k: v[1] for k, v in results.items()}
    if use_cache:
        _store_cache(key, plan)
    return plan
